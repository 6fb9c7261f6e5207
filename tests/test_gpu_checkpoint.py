"""Checkpoint and resume through the C ABI: an exported handle re-imports with identical
counters, coefficients and estimate, and by linearity a resumed stream ends where an
uninterrupted one does."""
import numpy as np
import pytest
import torch

import workloads as W
from tests.helpers import keys_u32, to_device_keys
from tests.test_abi import _blob

pytestmark = pytest.mark.gpu

if torch.cuda.is_available():
    import paper_2402_15953_amd as csk


@pytest.mark.parametrize("graph,m,d", [(W.chain(3), 1 << 16, 9), (W.fig3_query(), 1000, 5), (W.star(4), 4096, 3)])
def test_export_import_resume(graph, m, d):
    n = 60_000
    rels = [keys_u32(W.relation_keys(graph, k, n, "zipf", config=350, s=1.1, D=10 ** 5)) for k in range(graph.n_rel)]
    full = csk.Sketch(graph, m, d, 21)
    first = csk.Sketch(graph, m, d, 21)
    for k in range(graph.n_rel):
        kd = to_device_keys(rels[k])
        full.update(k, kd)
        first.update(k, kd[: n // 2])
    torch.cuda.synchronize()
    blob = first.export()
    resumed = csk.import_sketch(blob, graph)
    s1, b1 = first.coefficients()
    s2, b2 = resumed.coefficients()
    assert np.array_equal(s1, s2) and np.array_equal(b1, b2)
    for k in range(graph.n_rel):
        assert np.array_equal(resumed.read_sketch(k), first.read_sketch(k))
    assert resumed.estimate(reps=True) == first.estimate(reps=True)
    for k in range(graph.n_rel):
        resumed.update(k, to_device_keys(rels[k][n // 2:]))
    torch.cuda.synchronize()
    for k in range(graph.n_rel):
        assert np.array_equal(resumed.read_sketch(k), full.read_sketch(k))
    assert resumed.estimate() == full.estimate()
    assert resumed.export() == full.export()
    for s in (full, first, resumed):
        s.close()


def test_import_blob_written_from_the_documented_layout():
    """A blob assembled on the host from the header's layout imports to those counters."""
    m, d = 64, 2
    counters = [(i * 7919) % 2001 - 1000 for i in range(2 * d * m)]
    sk = csk.import_sketch(_blob(m=m, d=d, seed=5, counters=counters), W.single_join())
    got = np.concatenate([sk.read_sketch(0).ravel(), sk.read_sketch(1).ravel()])
    assert got.tolist() == counters
    ref = csk.Sketch(W.single_join(), m, d, 5)
    assert np.array_equal(sk.coefficients()[0], ref.coefficients()[0])
    sk.close()
    ref.close()
