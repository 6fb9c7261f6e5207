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


def test_tune_table_file_roundtrip(tmp_path):
    """The autotuner's table file: load, save, reload; a malformed file merges nothing."""
    import paper_2402_15953_amd as csk
    csk.tune_clear()
    assert csk.tune_count() == 0
    good = tmp_path / "tune.txt"
    good.write_text("csketch-tune 1\n"
                    "gfx950-256cu 65536 9 2 1 1 23 2 28 0 0.290000\n"
                    "gfx950-256cu 4096 5 1 1 0 16 1 0 0 0.010000\n")
    csk.tune_load(str(good))
    assert csk.tune_count() == 2
    out = tmp_path / "again.txt"
    csk.tune_save(str(out))
    lines = out.read_text().splitlines()
    assert lines[0] == "csketch-tune 1"
    assert sorted(lines[1:]) == sorted(good.read_text().splitlines()[1:])
    bad = tmp_path / "bad.txt"
    bad.write_text("csketch-tune 1\ngfx950-256cu 65536 9 2 1 1 23 7 28 0 0.29\n")   # strategy 7 does not exist
    with pytest.raises(csk.CsError) as e:
        csk.tune_load(str(bad))
    assert e.value.status == csk.CS_EINVAL
    assert csk.tune_count() == 2
    (tmp_path / "nohdr.txt").write_text("gfx950-256cu 65536 9 2 1 1 23 2 28 0 0.29\n")
    with pytest.raises(csk.CsError):
        csk.tune_load(str(tmp_path / "nohdr.txt"))
    csk.tune_clear()
    assert csk.tune_count() == 0


def _blob(m=64, d=2, seed=5, counters=None, version=1):
    """A checkpoint blob of the one-join query, built here from the documented layout."""
    import struct
    n_rel, n_attr, n_edge = 2, 2, 1
    nc = n_rel * d * m
    counters = list(range(nc)) if counters is None else counters
    body = b"CSKETCH1" + struct.pack("<6IQ", version, m, d, n_rel, n_attr, n_edge, seed)
    body += struct.pack("<2i", 0, 1) + struct.pack("<2i", 0, 1) + struct.pack("<%dq" % nc, *counters)
    h = 1469598103934665603
    for b in body:
        h = ((h ^ b) * 1099511628211) & ((1 << 64) - 1)
    return body + struct.pack("<Q", h)


def test_checkpoint_blob_validation_before_any_device_work():
    """cs_import refuses a malformed blob with CS_EINVAL before touching the device (so
    this runs without a GPU): wrong magic, version, length, checksum, header ranges."""
    import paper_2402_15953_amd as csk
    L = csk.lib()
    good = _blob()
    bad = [b"", b"NOTASKETCH" + good[10:], _blob(version=2), good[:-9] + good[-8:], good[:-1] + bytes([good[-1] ^ 1]),
           _blob(m=1, counters=[0] * 4), _blob(d=65, m=2, counters=[0] * 260)]
    corrupt = bytearray(good)
    corrupt[60] ^= 0xFF
    bad.append(bytes(corrupt))
    for blob in bad:
        h = ctypes.c_void_p()
        st = L.cs_import(blob, len(blob), ctypes.byref(h))
        assert st == csk.CS_EINVAL, (blob[:12], st)
        assert not h.value


def test_tune_table_batch_and_split_entries(tmp_path):
    """Batched-task (atomic 16, LDS segment 17, sort-reduce 18) and transform-split entries
    share the table file with plain-update entries (their own scope: same class fields,
    different entries) and are validated on load: chunk exponents 12..22, splits 2^S with
    S = 10..12 and S < log2 m <= 2S."""
    import paper_2402_15953_amd as csk
    csk.tune_clear()
    good = tmp_path / "tune.txt"
    good.write_text("csketch-tune 1\n"
                    "gfx950-256cu 65536 9 2 1 1 17 17 18 0 0.500000\n"
                    "gfx950-256cu 1024 5 1 1 1 12 16 16 0 0.010000\n"
                    "gfx950-256cu 262144 0 0 0 0 0 32 11 0 0.200000\n"
                    "gfx950-256cu 65536 9 2 1 1 17 2 28 0 0.290000\n"
                    "gfx950-256cu 4096 5 1 1 1 14 18 16 0 0.020000\n")
    csk.tune_load(str(good))
    assert csk.tune_count() == 5
    out = tmp_path / "again.txt"
    csk.tune_save(str(out))
    assert sorted(out.read_text().splitlines()[1:]) == sorted(good.read_text().splitlines()[1:])
    for bad_line in ("gfx950-256cu 262144 0 0 0 0 0 32 9 0 0.2",      # tile below 2^10
                     "gfx950-256cu 4096 0 0 0 0 0 32 10 0 0.2",        # one-pass length
                     "gfx950-256cu 1048576 0 0 0 0 0 32 13 0 0.2",     # tile above 2^12
                     "gfx950-256cu 100000 0 0 0 0 0 32 11 0 0.2",      # not a power of two
                     "gfx950-256cu 65536 9 2 1 1 17 17 30 0 0.5",      # chunk beyond 2^22
                     "gfx950-256cu 65536 9 2 1 1 17 33 18 0 0.5"):     # no such strategy code
        bad = tmp_path / "bad.txt"
        bad.write_text("csketch-tune 1\n" + bad_line + "\n")
        with pytest.raises(csk.CsError):
            csk.tune_load(str(bad))
    assert csk.tune_count() == 5
    csk.tune_clear()


def test_subquery_masks_validated_on_the_host():
    """cs_subq_create checks every sub-query (non-empty, joins of the graph, connected)
    and the per-relation limits before any device work: CS_EINVAL here without a GPU."""
    import paper_2402_15953_amd as csk
    import workloads as W
    L = csk.lib()

    def create(graph, masks):
        arr = (ctypes.c_uint32 * len(masks))(*masks)
        h = ctypes.c_void_p()
        st = L.cs_subq_create(ctypes.byref(csk._graph_struct(graph)), arr, len(masks), 1024, 2, 1, ctypes.byref(h))
        if h.value:
            L.cs_subq_destroy(h)
        return st

    for graph, masks in ((W.chain(4), [0b101]), (W.chain(4), [0]), (W.chain(4), [0b1000]),
                         (W.star(6), W.connected_subqueries(W.star(6)))):
        assert create(graph, masks) == csk.CS_EINVAL, (graph.name, masks)
    assert create(W.chain(5), W.connected_subqueries(W.chain(5))) in (csk.CS_OK, csk.CS_EDEVICE)
