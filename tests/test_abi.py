"""The C-ABI library loads and exports every entry point its header declares (CPU)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    names = set()
    for fn in os.listdir(os.path.join(ROOT, "include")):
        if fn.endswith(".h"):
            src = open(os.path.join(ROOT, "include", fn)).read()
            src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
            names |= set(re.findall(r"\b(cs_[a-z0-9_]+)\s*\(", src))
    return sorted(names)


def test_header_declares_entry_points():
    names = _declared()
    for must in ("cs_create", "cs_update", "cs_estimate", "cs_destroy"):
        assert must in names


def test_library_exports_every_declared_symbol():
    import paper_2402_15953_amd as csk
    L = csk.lib()
    missing = [n for n in _declared() if not hasattr(L, n)]
    assert not missing, missing
    assert sorted(set(csk.EXPORTED)) == sorted(set(n for n in _declared() if n in csk.EXPORTED))


def test_sketch_bytes_host_only():
    import paper_2402_15953_amd as csk
    import workloads as W
    assert csk.sketch_bytes(W.chain(3), 1 << 16, 9) == 3 * 9 * (1 << 16) * 8
    assert csk.sketch_bytes(W.single_join(), 1024, 5) == 2 * 5 * 1024 * 8


def test_binding_refuses_without_gpu():
    import torch
    import paper_2402_15953_amd as csk
    import workloads as W
    if torch.cuda.is_available():
        pytest.skip("GPU present")
    with pytest.raises(RuntimeError):
        csk.Sketch(W.chain(3), 1024, 5, 7)
