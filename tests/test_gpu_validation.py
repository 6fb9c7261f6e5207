"""Caller arrays the device cannot read (pageable host memory) are refused with
CS_EINVAL by every entry point that hands them to a kernel, before anything is
enqueued, and the handles keep working afterwards.  No kernel ever sees such a pointer:
the check runs on the host."""
import ctypes
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


def _einval(fn):
    with pytest.raises(csk.CsError) as e:
        fn()
    assert e.value.status == csk.CS_EINVAL, e.value


def test_pageable_arrays_refused_everywhere():
    graph = W.chain(3)
    n, m, d, seed = 5000, 1 << 12, 3, 4
    _say("validation", n, m, d)
    rels = [keys_u32(W.relation_keys(graph, k, n, "uniform", config=720, D=1000)) for k in range(3)]
    host_keys = [torch.from_numpy(np.ascontiguousarray(r).view(np.int32)) for r in rels]  # pageable
    dev_keys = [to_device_keys(r) for r in rels]
    host_w = torch.ones(n, dtype=torch.int64)
    L = csk.lib()

    sk = csk.Sketch(graph, m, d, seed)
    # cs_update: pageable keys; device keys with pageable weights
    _einval(lambda: csk._check(L.cs_update(sk.handle, 1, ctypes.c_void_p(host_keys[1].data_ptr()), None, n, None)))
    _einval(lambda: csk._check(L.cs_update(sk.handle, 0, ctypes.c_void_p(dev_keys[0].data_ptr()),
                                           ctypes.c_void_p(host_w.data_ptr()), n, None)))
    # cs_update_filtered: pageable attribute columns
    attrs = torch.zeros(n, 1, dtype=torch.int32)
    pred = (csk._Predicate * 1)(csk._Predicate(0, 0, 10))
    kept = ctypes.c_uint64()
    _einval(lambda: csk._check(L.cs_update_filtered(sk.handle, 0, ctypes.c_void_p(dev_keys[0].data_ptr()), None, n,
                                                    ctypes.c_void_p(attrs.data_ptr()), 1, pred, 1, 0, None,
                                                    ctypes.byref(kept))))
    # batched update and server submission
    b = csk.Batch()
    _einval(lambda: b.update([(sk, 0, host_keys[0], None, False)]))
    b.close()
    srv = csk.Server(n_streams=1, max_batch_items=16)
    q = srv.add_query(graph, m, d, seed)
    _einval(lambda: srv.submit_update(q, 0, host_keys[0]))
    _einval(lambda: srv.submit_update(q, 0, dev_keys[0], host_w))
    srv.close()
    # AMS baseline and per-attribute sketches
    ams = csk.AmsSketch(graph, 64, d, seed)
    _einval(lambda: ams.update(0, host_keys[0]))
    ams.close()
    ak = csk.AttrSketches(graph, m, d, seed)
    _einval(lambda: ak.update(1, host_keys[1]))
    ak.close()

    # nothing reached the counters, and the handle still works
    torch.cuda.synchronize()
    assert not any(sk.read_sketch(k).any() for k in range(3))
    for k in range(3):
        sk.update(k, dev_keys[k])
    torch.cuda.synchronize()
    _, _, ref = oracle_sketches(graph, rels, None, m, d, seed)
    for k in range(3):
        assert np.array_equal(sk.read_sketch(k), ref[k]), k
    sk.close()


def test_pinned_host_keys_accepted():
    """Pinned host memory is readable by the device: an update from it equals the one
    from device memory."""
    graph = W.single_join()
    n, m, d, seed = 20_000, 1 << 10, 5, 6
    rels = [keys_u32(W.relation_keys(graph, k, n, "zipf", config=721, s=1.1, D=5000)) for k in range(2)]
    a = csk.Sketch(graph, m, d, seed)
    b = csk.Sketch(graph, m, d, seed)
    for k in range(2):
        pin = torch.from_numpy(np.ascontiguousarray(rels[k]).view(np.int32)).pin_memory()
        a.update(k, to_device_keys(rels[k]))
        csk._check(csk.lib().cs_update(b.handle, k, ctypes.c_void_p(pin.data_ptr()), None, n, None))
        torch.cuda.synchronize()
    for k in range(2):
        assert np.array_equal(a.read_sketch(k), b.read_sketch(k))
    assert a.estimate() == b.estimate()
    a.close()
    b.close()
