"""The allocation-free update (cs_update_noalloc, static scratch array) through the C ABI:
its counters equal cs_update's bit for bit, over two calls in a row (the second with a
smaller input, so the array holds the first call's leftovers), for the 16-bit segmented,
int64 segmented and partition strategies; a geometry the array cannot hold is refused."""
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


CASES = [
    # graph, m, d, sizes of the two calls, weights, D
    (W.chain(3), 1 << 16, 9, (300_000, 70_001), None, 10 ** 6),
    (W.chain(5), 1 << 18, 15, (1 << 20, 123_457), None, 10 ** 7),
    (W.chain(3), 1 << 18, 5, (200_000, 50_003), "pm1", 10 ** 7),
    (W.star(4), 4096, 7, (90_000, 20_011), "big", 10 ** 4),
    (W.single_join(), 1024, 5, (100_000, 999), None, 10 ** 4),
]


def _weights(kind, n, seed):
    if kind is None:
        return None
    if kind == "pm1":
        return W.turnstile_weights(n, 0.1, seed=seed).cuda()
    return W.random_weights(n, -2 ** 62, 2 ** 62, seed=seed).cuda()


@pytest.mark.parametrize("case", range(len(CASES)))
def test_noalloc_equals_update(case):
    graph, m, d, sizes, wk, D = CASES[case]
    _say("noalloc", case, graph.name, m, d, sizes, wk)
    seed = 40 + case
    sa = csk.Sketch(graph, m, d, seed)   # allocation-free entry point
    sb = csk.Sketch(graph, m, d, seed)   # cs_update
    for call, n in enumerate(sizes):
        for k in range(graph.n_rel):
            keys = to_device_keys(keys_u32(W.relation_keys(graph, k, n, "zipf", config=900 + 10 * case + call,
                                                           s=1.1, D=D)))
            w = _weights(wk, n, seed=100 * case + 10 * call + k)
            unit = wk == "pm1"
            sa.update_noalloc(k, keys, w, unit_weights=unit)
            sb.update(k, keys, w, unit_weights=unit)
        torch.cuda.synchronize()
        for k in range(graph.n_rel):
            assert np.array_equal(sa.read_sketch(k), sb.read_sketch(k)), (case, call, k)
    assert sa.estimate() == sb.estimate()
    sa.close()
    sb.close()


def test_noalloc_refuses_what_the_array_cannot_hold():
    """General weights at m = 2^18, d = 64: the int64 segmented strategy needs d * m * 8 =
    128 MiB of partial sums for one chunk, beyond the 64 MiB array: CS_EINVAL, nothing
    enqueued (the counters stay zero), and the handle keeps working."""
    assert csk.lib().cs_update_noalloc_scratch_bytes() == 64 << 20
    g = W.single_join()
    sk = csk.Sketch(g, 1 << 18, 64, 3)
    n = 10_000
    keys = to_device_keys(keys_u32(W.relation_keys(g, 0, n, "uniform", config=990, D=10 ** 6)))
    w = W.random_weights(n, -100, 100, seed=5).cuda()
    with pytest.raises(csk.CsError) as e:
        sk.update_noalloc(0, keys, w)
    assert e.value.status == csk.CS_EINVAL
    torch.cuda.synchronize()
    assert not sk.read_sketch(0).any()
    sk.update_noalloc(0, keys, torch.ones(n, dtype=torch.int64, device="cuda"), unit_weights=True)
    ref = csk.Sketch(g, 1 << 18, 64, 3)
    ref.update(0, keys, torch.ones(n, dtype=torch.int64, device="cuda"), unit_weights=True)
    torch.cuda.synchronize()
    assert np.array_equal(sk.read_sketch(0), ref.read_sketch(0))
    sk.close()
    ref.close()
