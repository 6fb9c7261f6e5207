"""Python binding of libcsketch (MI355X convolution Count sketches).

Argument marshalling only: every step of the update and the estimate runs in the HIP
library.  Device buffers are torch tensors on the current HIP device; streams are
torch streams.  There is no CPU fallback: without the built library or a GPU, the
calls raise.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional, Sequence

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libcsketch.so")

CS_OK, CS_EINVAL, CS_EGRAPH, CS_ENOMEM, CS_EDEVICE, CS_EBUSY, CS_ERANGE = range(7)
UPDATE_AUTO, UPDATE_GLOBAL_ATOMIC, UPDATE_LDS_PRIVATE, UPDATE_WAVE_AGGREGATE, UPDATE_PARTITION = range(5)
UPDATE_UNIT_WEIGHTS = 1
UPDATE_NO_COMPACT = 2
UPDATE_NO_COUNTERS16 = 4
UPDATE_TEST_FULL_REDUCTION = 8
PLAN_DOT, PLAN_SPECTRAL, PLAN_GENERAL = 1, 2, 3

EXPORTED = [
    "cs_create", "cs_destroy", "cs_sketch_bytes", "cs_get_info", "cs_last_error",
    "cs_update", "cs_update_ex", "cs_update_timed", "cs_update_noalloc", "cs_update_noalloc_scratch_bytes",
    "cs_k0_horner", "cs_k0_stream_read",
    "cs_update_filtered", "cs_estimate", "cs_reset", "cs_merge", "cs_read_sketch",
    "cs_sketch_device_ptr", "cs_read_coeffs", "cs_read_components",
    "cs_timer_create", "cs_timer_record", "cs_timer_elapsed", "cs_timer_destroy",
    "cs_tune_update", "cs_tune_clear", "cs_tune_save", "cs_tune_load", "cs_tune_count",
    "cs_tune_batch_update", "cs_tune_transform",
    "cs_batch_create", "cs_batch_destroy", "cs_batch_update", "cs_batch_capture", "cs_batch_replay",
    "cs_batch_estimate", "cs_batch_stats", "cs_batch_task_counts",
    "cs_server_create", "cs_server_destroy", "cs_server_add_query", "cs_server_remove_query",
    "cs_server_sketch", "cs_server_submit_update", "cs_server_submit_estimate", "cs_server_poll",
    "cs_server_drain", "cs_server_stats",
    "cs_ams_create", "cs_ams_destroy", "cs_ams_update", "cs_ams_reset", "cs_ams_estimate", "cs_ams_read",
    "cs_ams_coefficients",
    "cs_attr_create", "cs_attr_destroy", "cs_attr_update", "cs_attr_reset", "cs_attr_estimate_join",
    "cs_attr_read", "cs_attr_coefficients",
    "cs_subq_create", "cs_subq_destroy", "cs_subq_update", "cs_subq_reset", "cs_subq_estimate",
    "cs_subq_estimate_all", "cs_subq_layout", "cs_subq_read", "cs_subq_coefficients",
    "cs_export", "cs_import", "cs_estimate_async",
]


class CsError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"csketch status {status}: {msg}")
        self.status = status


class _Graph(ctypes.Structure):
    _fields_ = [("n_rel", ctypes.c_int32), ("n_attr", ctypes.c_int32),
                ("attr_rel", ctypes.POINTER(ctypes.c_int32)), ("n_edge", ctypes.c_int32),
                ("edges", ctypes.POINTER(ctypes.c_int32))]


class _AmsEstimate(ctypes.Structure):
    _fields_ = [("value", ctypes.c_double), ("num_lo", ctypes.c_int64), ("num_hi", ctypes.c_int64),
                ("exact", ctypes.c_int32), ("median_rep", ctypes.c_int32)]


class _Estimate(ctypes.Structure):
    _fields_ = [("value", ctypes.c_double), ("value_i64", ctypes.c_int64), ("exact", ctypes.c_int32),
                ("fits_i64", ctypes.c_int32), ("d", ctypes.c_int32), ("n_modular", ctypes.c_int32)]


class _Reps(ctypes.Structure):
    _fields_ = [("value", ctypes.c_void_p), ("lo", ctypes.c_void_p), ("hi", ctypes.c_void_p),
                ("exact", ctypes.c_void_p), ("bound", ctypes.c_void_p)]


MAX_PREDICATES = 8


class _Predicate(ctypes.Structure):
    _fields_ = [("column", ctypes.c_int32), ("lo", ctypes.c_uint32), ("hi", ctypes.c_uint32)]


class _TuneCand(ctypes.Structure):
    _fields_ = [("strategy", ctypes.c_int32), ("grid_blocks", ctypes.c_int32), ("flags", ctypes.c_int32),
                ("valid", ctypes.c_int32), ("ms", ctypes.c_float)]


TUNE_MAX_CANDIDATES = 16


class _TuneReport(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32), ("best", ctypes.c_int32), ("cand", _TuneCand * TUNE_MAX_CANDIDATES)]


class _TuneBatchReport(ctypes.Structure):
    _fields_ = [("classes", ctypes.c_int32), ("rejected", ctypes.c_int32), ("rule_ms", ctypes.c_float),
                ("tuned_ms", ctypes.c_float)]


class _Item(ctypes.Structure):
    _fields_ = [("sketch", ctypes.c_void_p), ("rel", ctypes.c_int32), ("flags", ctypes.c_int32),
                ("keys", ctypes.c_void_p), ("weights", ctypes.c_void_p), ("n", ctypes.c_uint64)]


class _ServerConfig(ctypes.Structure):
    _fields_ = [("memory_budget", ctypes.c_uint64), ("n_streams", ctypes.c_int32),
                ("max_batch_items", ctypes.c_int32), ("max_pending", ctypes.c_int32), ("reserved", ctypes.c_int32)]


class _Completion(ctypes.Structure):
    _fields_ = [("ticket", ctypes.c_uint64), ("qid", ctypes.c_int32), ("kind", ctypes.c_int32),
                ("status", ctypes.c_int32), ("reserved", ctypes.c_int32), ("submit_us", ctypes.c_double),
                ("start_us", ctypes.c_double), ("done_us", ctypes.c_double), ("estimate", _Estimate)]


class _ServerStats(ctypes.Structure):
    _fields_ = [("submitted", ctypes.c_uint64), ("completed", ctypes.c_uint64), ("used_bytes", ctypes.c_uint64),
                ("update_launches", ctypes.c_uint64), ("estimate_batches", ctypes.c_uint64),
                ("epochs", ctypes.c_uint64), ("live_queries", ctypes.c_int32), ("reserved", ctypes.c_int32)]


class _Info(ctypes.Structure):
    _fields_ = [("n_rel", ctypes.c_int32), ("n_attr", ctypes.c_int32), ("n_edge", ctypes.c_int32),
                ("n_comp", ctypes.c_int32), ("m", ctypes.c_uint32), ("d", ctypes.c_uint32),
                ("plan", ctypes.c_int32), ("device", ctypes.c_int32), ("counter_bytes", ctypes.c_uint64),
                ("workspace_bytes", ctypes.c_uint64)]


_lib = None


def lib() -> ctypes.CDLL:
    """Load libcsketch.so (building it first only if it has never been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            from . import build as _b
            _b.build()
        L = ctypes.CDLL(LIB_PATH)
        vp, i32, u32, u64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_uint32, ctypes.c_uint64
        L.cs_create.argtypes = [ctypes.POINTER(_Graph), u32, u32, u64, ctypes.POINTER(vp)]
        L.cs_destroy.argtypes = [vp]
        L.cs_sketch_bytes.argtypes = [ctypes.POINTER(_Graph), u32, u32]
        L.cs_sketch_bytes.restype = u64
        L.cs_get_info.argtypes = [vp, ctypes.POINTER(_Info)]
        L.cs_last_error.restype = ctypes.c_char_p
        L.cs_update.argtypes = [vp, i32, vp, vp, u64, vp]
        L.cs_update_ex.argtypes = [vp, i32, vp, vp, u64, vp, i32, i32, i32]
        L.cs_update_timed.argtypes = [vp, i32, vp, vp, u64, vp, i32, i32, i32, vp, vp]
        L.cs_update_noalloc.argtypes = [vp, i32, vp, vp, u64, i32, vp]
        L.cs_k0_horner.argtypes = [u64, ctypes.POINTER(ctypes.c_double)]
        L.cs_k0_stream_read.argtypes = [vp, u64, i32, ctypes.POINTER(ctypes.c_double)]
        L.cs_update_noalloc_scratch_bytes.argtypes = []
        L.cs_update_noalloc_scratch_bytes.restype = ctypes.c_size_t
        L.cs_update_filtered.argtypes = [vp, i32, vp, vp, u64, vp, i32, ctypes.POINTER(_Predicate), i32, i32, vp,
                                         ctypes.POINTER(u64)]
        L.cs_estimate.argtypes = [vp, vp, ctypes.POINTER(_Estimate), ctypes.POINTER(_Reps)]
        L.cs_reset.argtypes = [vp, vp]
        L.cs_merge.argtypes = [vp, vp, vp]
        L.cs_read_sketch.argtypes = [vp, i32, vp]
        L.cs_sketch_device_ptr.argtypes = [vp, i32, ctypes.POINTER(vp)]
        L.cs_read_coeffs.argtypes = [vp, vp, vp]
        L.cs_read_components.argtypes = [vp, vp]
        L.cs_timer_create.argtypes = [ctypes.POINTER(vp)]
        L.cs_timer_record.argtypes = [vp, vp]
        L.cs_timer_elapsed.argtypes = [vp, vp, ctypes.POINTER(ctypes.c_float)]
        L.cs_timer_destroy.argtypes = [vp]
        L.cs_tune_update.argtypes = [vp, i32, vp, vp, u64, vp, i32, ctypes.POINTER(_TuneReport)]
        L.cs_tune_clear.argtypes = []
        L.cs_tune_save.argtypes = [ctypes.c_char_p]
        L.cs_tune_load.argtypes = [ctypes.c_char_p]
        L.cs_tune_count.argtypes = [ctypes.POINTER(ctypes.c_int32)]
        L.cs_tune_batch_update.argtypes = [vp, vp, i32, vp, ctypes.POINTER(_TuneBatchReport)]
        L.cs_tune_transform.argtypes = [i32, i32, vp, ctypes.POINTER(_TuneReport)]
        L.cs_batch_create.argtypes = [ctypes.POINTER(vp)]
        L.cs_batch_destroy.argtypes = [vp]
        L.cs_batch_update.argtypes = [vp, ctypes.POINTER(_Item), i32, vp]
        L.cs_batch_capture.argtypes = [vp, ctypes.POINTER(_Item), i32, vp]
        L.cs_batch_replay.argtypes = [vp, vp]
        L.cs_batch_estimate.argtypes = [vp, ctypes.POINTER(vp), i32, vp, ctypes.POINTER(_Estimate),
                                        ctypes.POINTER(_Reps)]
        L.cs_batch_stats.argtypes = [vp, ctypes.POINTER(u64), ctypes.POINTER(u64)]
        L.cs_batch_task_counts.argtypes = [vp, ctypes.POINTER(u64), ctypes.POINTER(u64), ctypes.POINTER(u64)]
        L.cs_server_create.argtypes = [ctypes.POINTER(_ServerConfig), ctypes.POINTER(vp)]
        L.cs_server_destroy.argtypes = [vp]
        L.cs_server_add_query.argtypes = [vp, ctypes.POINTER(_Graph), u32, u32, u64, ctypes.POINTER(i32)]
        L.cs_server_remove_query.argtypes = [vp, i32]
        L.cs_server_sketch.argtypes = [vp, i32, ctypes.POINTER(vp)]
        L.cs_server_submit_update.argtypes = [vp, i32, i32, vp, vp, u64, i32, ctypes.POINTER(u64)]
        L.cs_server_submit_estimate.argtypes = [vp, i32, ctypes.POINTER(u64)]
        L.cs_server_poll.argtypes = [vp, ctypes.POINTER(_Completion), i32, ctypes.POINTER(i32)]
        L.cs_server_drain.argtypes = [vp]
        L.cs_server_stats.argtypes = [vp, ctypes.POINTER(_ServerStats)]
        L.cs_ams_create.argtypes = [ctypes.POINTER(_Graph), u32, u32, u64, ctypes.POINTER(vp)]
        L.cs_ams_destroy.argtypes = [vp]
        L.cs_ams_update.argtypes = [vp, i32, vp, vp, u64, vp]
        L.cs_ams_reset.argtypes = [vp, vp]
        L.cs_ams_estimate.argtypes = [vp, vp, ctypes.POINTER(_AmsEstimate), vp, vp, vp]
        L.cs_ams_read.argtypes = [vp, i32, vp]
        L.cs_ams_coefficients.argtypes = [vp, vp]
        L.cs_attr_create.argtypes = [ctypes.POINTER(_Graph), u32, u32, u64, ctypes.POINTER(vp)]
        L.cs_attr_destroy.argtypes = [vp]
        L.cs_attr_update.argtypes = [vp, i32, vp, vp, u64, i32, vp]
        L.cs_attr_reset.argtypes = [vp, vp]
        L.cs_attr_estimate_join.argtypes = [vp, i32, i32, vp, ctypes.POINTER(_Estimate), ctypes.POINTER(_Reps)]
        L.cs_attr_read.argtypes = [vp, i32, vp]
        L.cs_attr_coefficients.argtypes = [vp, vp, vp]
        L.cs_subq_create.argtypes = [ctypes.POINTER(_Graph), vp, i32, u32, u32, u64, ctypes.POINTER(vp)]
        L.cs_subq_destroy.argtypes = [vp]
        L.cs_subq_update.argtypes = [vp, i32, vp, vp, u64, i32, vp]
        L.cs_subq_reset.argtypes = [vp, vp]
        L.cs_subq_estimate.argtypes = [vp, i32, vp, ctypes.POINTER(_Estimate), ctypes.POINTER(_Reps)]
        L.cs_subq_estimate_all.argtypes = [vp, vp, vp]
        L.cs_subq_layout.argtypes = [vp, vp, vp]
        L.cs_subq_read.argtypes = [vp, i32, vp]
        L.cs_subq_coefficients.argtypes = [vp, vp, vp, vp]
        L.cs_export.argtypes = [vp, vp, ctypes.c_size_t, ctypes.POINTER(ctypes.c_size_t)]
        L.cs_import.argtypes = [vp, ctypes.c_size_t, ctypes.POINTER(vp)]
        L.cs_estimate_async.argtypes = [vp, vp, vp]
        _lib = L
    return _lib


def _check(status: int):
    if status != CS_OK:
        raise CsError(status, lib().cs_last_error().decode())


def _graph_struct(graph):
    attr = (ctypes.c_int32 * len(graph.attr_rel))(*graph.attr_rel)
    flat = [x for e in graph.edges for x in e]
    edges = (ctypes.c_int32 * max(1, len(flat)))(*flat)
    g = _Graph(int(graph.n_rel), len(graph.attr_rel), attr, len(graph.edges), edges)
    g._keep = (attr, edges)
    return g


def _stream_ptr(stream):
    if stream is None:
        import torch
        return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    if isinstance(stream, int):
        return ctypes.c_void_p(stream)
    return ctypes.c_void_p(stream.cuda_stream)


def _event_ptr(ev):
    """Raw hipEvent_t of a Timer or a torch.cuda.Event (created on first use), or None."""
    if ev is None:
        return None
    if isinstance(ev, Timer):
        return ev.handle
    if not ev.cuda_event:
        ev.record()   # torch creates the event lazily, on its first record
    return ctypes.c_void_p(ev.cuda_event)


class Timer:
    """A timing event without the system-scope fence (cs_timer_*): recording it does not
    write back caches in the middle of the timed work."""

    def __init__(self):
        h = ctypes.c_void_p()
        _check(lib().cs_timer_create(ctypes.byref(h)))
        self.handle = h

    def record(self, stream=None):
        _check(lib().cs_timer_record(self.handle, _stream_ptr(stream)))

    def elapsed_ms(self, stop: "Timer") -> float:
        ms = ctypes.c_float()
        _check(lib().cs_timer_elapsed(self.handle, stop.handle, ctypes.byref(ms)))
        return float(ms.value)

    def close(self):
        if getattr(self, "handle", None):
            lib().cs_timer_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _reps_struct(d):
    arrs = dict(value=np.zeros(d, np.float64), lo=np.zeros(d, np.int64), hi=np.zeros(d, np.int64),
                exact=np.zeros(d, np.int32), bound=np.zeros(d, np.float64))
    rp = _Reps(*(a.ctypes.data for a in (arrs["value"], arrs["lo"], arrs["hi"], arrs["exact"], arrs["bound"])))
    return rp, arrs


def _estimate_dict(e, arrs):
    out = dict(value=e.value, value_i64=e.value_i64 if e.fits_i64 else None, exact=bool(e.exact),
               d=e.d, n_modular=e.n_modular)
    if arrs is not None:
        ints = []
        for t in range(len(arrs["value"])):
            if arrs["exact"][t]:
                ints.append((int(arrs["hi"][t]) << 64) | (int(arrs["lo"][t]) & ((1 << 64) - 1)))
            else:
                ints.append(None)
        out.update(rep_values=arrs["value"].tolist(), rep_ints=ints, rep_bounds=arrs["bound"].tolist())
    return out


STRATEGY_NAMES = {UPDATE_GLOBAL_ATOMIC: "global_atomic", UPDATE_LDS_PRIVATE: "lds_segmented",
                  UPDATE_WAVE_AGGREGATE: "wave_aggregate", UPDATE_PARTITION: "partition"}


def tune_update(sketch: "Sketch", rel: int, keys, weights=None, unit_weights: bool = False, stream=None) -> dict:
    """Autotune the update for this handle's class on these tuples (cs_tune_update);
    returns the candidates with their median times and the chosen one."""
    n = keys.shape[0]
    rep = _TuneReport()
    wp = None if weights is None else ctypes.c_void_p(weights.data_ptr())
    _check(lib().cs_tune_update(sketch.handle, int(rel), ctypes.c_void_p(keys.data_ptr()), wp, int(n),
                                _stream_ptr(stream), UPDATE_UNIT_WEIGHTS if unit_weights else 0, ctypes.byref(rep)))
    cands = [dict(strategy=STRATEGY_NAMES.get(c.strategy, c.strategy), grid=c.grid_blocks, flags=c.flags,
                  valid=int(c.valid), ms=float(c.ms)) for c in rep.cand[:rep.n]]
    return {"candidates": cands, "best": cands[rep.best], "best_index": rep.best}


TUNE_BATCH_ATOMIC, TUNE_BATCH_SEGMENT, TUNE_BATCH_SORT, TUNE_TRANSFORM_SPLIT = 16, 17, 18, 32


def tune_transform(log2m: int, n_vec: int = 64, stream=None) -> dict:
    """Autotune the row length of the two-pass transforms of length 2^log2m
    (cs_tune_transform); returns each split's median time and the chosen one."""
    rep = _TuneReport()
    _check(lib().cs_tune_transform(int(log2m), int(n_vec), _stream_ptr(stream), ctypes.byref(rep)))
    cands = [dict(split=c.grid_blocks, valid=int(c.valid), ms=float(c.ms)) for c in rep.cand[:rep.n]]
    return {"candidates": cands, "best": cands[rep.best], "best_index": rep.best}


def tune_clear():
    _check(lib().cs_tune_clear())


def tune_save(path: str):
    _check(lib().cs_tune_save(str(path).encode()))


def tune_load(path: str):
    _check(lib().cs_tune_load(str(path).encode()))


def tune_count() -> int:
    n = ctypes.c_int32()
    _check(lib().cs_tune_count(ctypes.byref(n)))
    return n.value


def k0_horner(iters: int = 1 << 14) -> float:
    """Horner steps per second of a kernel made of nothing but independent steps."""
    r = ctypes.c_double()
    _check(lib().cs_k0_horner(int(iters), ctypes.byref(r)))
    return r.value


def k0_stream_read(buf, passes: int = 5) -> float:
    """Bytes per second of a kernel streaming the device tensor `buf` (read only)."""
    r = ctypes.c_double()
    _check(lib().cs_k0_stream_read(ctypes.c_void_p(buf.data_ptr()), int(buf.numel() * buf.element_size()),
                                   int(passes), ctypes.byref(r)))
    return r.value


def sketch_bytes(graph, m: int, d: int) -> int:
    return int(lib().cs_sketch_bytes(ctypes.byref(_graph_struct(graph)), m, d))


class Sketch:
    """The d x m int64 sketches of every relation of one join query."""

    def __init__(self, graph, m: int, d: int, seed: int):
        import torch
        if not torch.cuda.is_available():
            raise RuntimeError("csketch needs a HIP GPU; there is no CPU fallback")
        self.graph = graph
        self.m, self.d, self.seed = int(m), int(d), int(seed)
        h = ctypes.c_void_p()
        _check(lib().cs_create(ctypes.byref(_graph_struct(graph)), self.m, self.d, self.seed, ctypes.byref(h)))
        self._h = h

    def close(self):
        if getattr(self, "_h", None):
            lib().cs_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def handle(self):
        return self._h

    def info(self) -> dict:
        i = _Info()
        _check(lib().cs_get_info(self._h, ctypes.byref(i)))
        return {f: getattr(i, f) for f, _ in _Info._fields_}

    def update(self, rel: int, keys, weights=None, stream=None, strategy: int = UPDATE_AUTO, grid: int = 0,
               unit_weights: bool = False, compact: bool = True, counters16: bool = True, timing=None,
               extra_flags: int = 0):
        """keys: device int32/uint32 tensor [n, a_rel] (or [n] for one column), contiguous;
        weights: device int64 tensor [n] or None; unit_weights: every weight is +-1;
        timing: optional (start, stop) torch.cuda.Event pair recorded around the hashing
        kernel (cs_update_timed)."""
        import torch
        if keys.dtype not in (torch.int32, torch.uint32) or not keys.is_cuda or not keys.is_contiguous():
            raise TypeError("keys must be a contiguous int32/uint32 device tensor")
        n = keys.shape[0]
        wp = None
        if weights is not None:
            if weights.dtype != torch.int64 or not weights.is_cuda or not weights.is_contiguous() \
                    or weights.shape[0] != n:
                raise TypeError("weights must be a contiguous int64 device tensor of length n")
            wp = ctypes.c_void_p(weights.data_ptr())
        flags = ((UPDATE_UNIT_WEIGHTS if unit_weights else 0) | (0 if compact else UPDATE_NO_COMPACT)
                 | (0 if counters16 else UPDATE_NO_COUNTERS16) | int(extra_flags))
        if timing is None:
            _check(lib().cs_update_ex(self._h, int(rel), ctypes.c_void_p(keys.data_ptr()), wp, int(n),
                                      _stream_ptr(stream), int(strategy), int(grid), flags))
        else:
            e0, e1 = _event_ptr(timing[0]), _event_ptr(timing[1])
            _check(lib().cs_update_timed(self._h, int(rel), ctypes.c_void_p(keys.data_ptr()), wp, int(n),
                                         _stream_ptr(stream), int(strategy), int(grid), flags, e0, e1))

    def update_noalloc(self, rel: int, keys, weights=None, stream=None, unit_weights: bool = False):
        """cs_update_noalloc: the automatic update with the library's static scratch array
        (nothing is allocated); same arguments and counters as update()."""
        import torch
        if keys.dtype not in (torch.int32, torch.uint32) or not keys.is_cuda or not keys.is_contiguous():
            raise TypeError("keys must be a contiguous int32/uint32 device tensor")
        n = keys.shape[0]
        wp = None
        if weights is not None:
            if weights.dtype != torch.int64 or not weights.is_cuda or not weights.is_contiguous() \
                    or weights.shape[0] != n:
                raise TypeError("weights must be a contiguous int64 device tensor of length n")
            wp = ctypes.c_void_p(weights.data_ptr())
        _check(lib().cs_update_noalloc(self._h, int(rel), ctypes.c_void_p(keys.data_ptr()), wp, int(n),
                                       UPDATE_UNIT_WEIGHTS if unit_weights else 0, _stream_ptr(stream)))

    def update_filtered(self, rel: int, keys, attrs, predicates, weights=None, stream=None,
                        unit_weights: bool = False, count: bool = True):
        """Stream only the tuples whose attrs satisfy every (column, lo, hi) predicate
        (lo <= attrs[i][column] <= hi); attrs: device int32/uint32 tensor [n, n_attrs].
        count: return the number of tuples kept (the call then waits for it); with
        count=False the call is asynchronous and returns None."""
        import torch
        if keys.dtype not in (torch.int32, torch.uint32) or not keys.is_cuda or not keys.is_contiguous():
            raise TypeError("keys must be a contiguous int32/uint32 device tensor")
        n = keys.shape[0]
        preds = list(predicates)
        arr = (_Predicate * max(1, len(preds)))(*[_Predicate(int(c), int(lo), int(hi)) for c, lo, hi in preds])
        ap, n_attrs = None, 0
        if attrs is not None:
            if attrs.dtype not in (torch.int32, torch.uint32) or not attrs.is_cuda or not attrs.is_contiguous() \
                    or attrs.shape[0] != n:
                raise TypeError("attrs must be a contiguous int32/uint32 device tensor [n, n_attrs]")
            ap = ctypes.c_void_p(attrs.data_ptr())
            n_attrs = 1 if attrs.dim() == 1 else int(attrs.shape[1])
        wp = None if weights is None else ctypes.c_void_p(weights.data_ptr())
        kept = ctypes.c_uint64()
        _check(lib().cs_update_filtered(self._h, int(rel), ctypes.c_void_p(keys.data_ptr()), wp, int(n), ap, n_attrs,
                                        arr, len(preds), UPDATE_UNIT_WEIGHTS if unit_weights else 0,
                                        _stream_ptr(stream), ctypes.byref(kept) if count else None))
        return kept.value if count else None

    def estimate(self, stream=None, reps: bool = False) -> dict:
        e = _Estimate()
        rp, arrs = _reps_struct(self.d) if reps else (None, None)
        _check(lib().cs_estimate(self._h, _stream_ptr(stream), ctypes.byref(e),
                                 ctypes.byref(rp) if rp is not None else None))
        return _estimate_dict(e, arrs)

    def estimate_async(self, out_ptr: int, stream=None):
        """Enqueue an estimate whose cs_estimate_t lands at out_ptr (device memory or
        pinned host memory) once the stream passes it; see read_estimate."""
        _check(lib().cs_estimate_async(self._h, _stream_ptr(stream), ctypes.c_void_p(out_ptr)))

    def reset(self, stream=None):
        _check(lib().cs_reset(self._h, _stream_ptr(stream)))

    def merge_from(self, other: "Sketch", stream=None):
        _check(lib().cs_merge(self._h, other._h, _stream_ptr(stream)))

    def read_sketch(self, rel: int) -> np.ndarray:
        out = np.zeros((self.d, self.m), dtype=np.int64)
        _check(lib().cs_read_sketch(self._h, int(rel), out.ctypes.data))
        return out

    def export(self) -> bytes:
        """Checkpoint blob (cs_export): graph, m, d, seed and counters."""
        need = ctypes.c_size_t()
        _check(lib().cs_export(self._h, None, 0, ctypes.byref(need)))
        buf = ctypes.create_string_buffer(need.value)
        _check(lib().cs_export(self._h, buf, need.value, ctypes.byref(need)))
        return buf.raw

    def device_ptr(self, rel: int) -> int:
        p = ctypes.c_void_p()
        _check(lib().cs_sketch_device_ptr(self._h, int(rel), ctypes.byref(p)))
        return p.value

    def coefficients(self):
        E, Q = len(self.graph.edges), self.info()["n_comp"]
        s = np.zeros((self.d, E, 4), dtype=np.uint64)
        b = np.zeros((self.d, Q, 2), dtype=np.uint64)
        _check(lib().cs_read_coeffs(self._h, s.ctypes.data, b.ctypes.data))
        return s, b

    def components(self) -> list:
        out = np.zeros(len(self.graph.attr_rel), dtype=np.int32)
        _check(lib().cs_read_components(self._h, out.ctypes.data))
        return out.tolist()


class Batch:
    """Batched updates (one persistent launch) and estimates over many Sketch handles."""

    def __init__(self):
        import torch
        if not torch.cuda.is_available():
            raise RuntimeError("csketch needs a HIP GPU; there is no CPU fallback")
        b = ctypes.c_void_p()
        _check(lib().cs_batch_create(ctypes.byref(b)))
        self._b = b
        self._keep = None

    def close(self):
        if getattr(self, "_b", None):
            lib().cs_batch_destroy(self._b)
            self._b = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @staticmethod
    def _items(items):
        """items: iterable of (sketch, rel, keys, weights_or_None, unit_weights)."""
        items = list(items)
        arr = (_Item * max(1, len(items)))()
        for i, (sk, rel, keys, w, unit) in enumerate(items):
            arr[i] = _Item(sk.handle.value, int(rel), UPDATE_UNIT_WEIGHTS if unit else 0,
                           keys.data_ptr(), None if w is None else w.data_ptr(), int(keys.shape[0]))
        return arr, len(items)

    def update(self, items, stream=None):
        arr, n = self._items(items)
        _check(lib().cs_batch_update(self._b, arr, n, _stream_ptr(stream)))

    def capture(self, items, stream=None):
        arr, n = self._items(items)
        _check(lib().cs_batch_capture(self._b, arr, n, _stream_ptr(stream)))

    def replay(self, stream=None):
        _check(lib().cs_batch_replay(self._b, _stream_ptr(stream)))

    def tune(self, items, stream=None) -> dict:
        """Autotune the task choice of every item class in this batch (cs_tune_batch_update)."""
        arr, n = self._items(items)
        rep = _TuneBatchReport()
        _check(lib().cs_tune_batch_update(self._b, arr, n, _stream_ptr(stream), ctypes.byref(rep)))
        return {"classes": rep.classes, "rejected": rep.rejected, "rule_ms": rep.rule_ms, "tuned_ms": rep.tuned_ms}

    def stats(self):
        a, b, c = ctypes.c_uint64(), ctypes.c_uint64(), ctypes.c_uint64()
        _check(lib().cs_batch_task_counts(self._b, ctypes.byref(a), ctypes.byref(b), ctypes.byref(c)))
        return {"tasks_atomic": a.value, "tasks_segment": b.value, "tasks_sort_reduce": c.value}

    def estimate(self, sketches, stream=None, reps: bool = False):
        sketches = list(sketches)
        n = len(sketches)
        hs = (ctypes.c_void_p * max(1, n))(*[s.handle.value for s in sketches])
        outs = (_Estimate * max(1, n))()
        rps, arrs = None, None
        if reps:
            pairs = [_reps_struct(s.d) for s in sketches]
            rps = (_Reps * n)(*[p[0] for p in pairs])
            arrs = [p[1] for p in pairs]
        _check(lib().cs_batch_estimate(self._b, hs, n, _stream_ptr(stream), outs, rps))
        return [_estimate_dict(outs[i], arrs[i] if arrs else None) for i in range(n)]


class _Borrowed(Sketch):
    """A live query's handle owned by a Server (read-only use)."""

    def __init__(self, h, graph, m, d, seed):  # noqa: D401 - no cs_create
        self._h = h
        self.graph, self.m, self.d, self.seed = graph, m, d, seed

    def close(self):
        self._h = None


class Server:
    """Serving loop: live sketches in HBM, update batches and estimates as they arrive."""

    def __init__(self, memory_budget: int = 0, n_streams: int = 2, max_batch_items: int = 4096,
                 max_pending: int = 0):
        import torch
        if not torch.cuda.is_available():
            raise RuntimeError("csketch needs a HIP GPU; there is no CPU fallback")
        cfg = _ServerConfig(int(memory_budget), int(n_streams), int(max_batch_items), int(max_pending), 0)
        s = ctypes.c_void_p()
        _check(lib().cs_server_create(ctypes.byref(cfg), ctypes.byref(s)))
        self._s = s
        self._queries = {}

    def close(self):
        if getattr(self, "_s", None):
            lib().cs_server_destroy(self._s)
            self._s = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def add_query(self, graph, m: int, d: int, seed: int) -> int:
        q = ctypes.c_int32()
        _check(lib().cs_server_add_query(self._s, ctypes.byref(_graph_struct(graph)), int(m), int(d), int(seed),
                                         ctypes.byref(q)))
        self._queries[q.value] = (graph, int(m), int(d), int(seed))
        return q.value

    def remove_query(self, qid: int):
        _check(lib().cs_server_remove_query(self._s, int(qid)))
        self._queries.pop(qid, None)

    def sketch(self, qid: int) -> Sketch:
        h = ctypes.c_void_p()
        _check(lib().cs_server_sketch(self._s, int(qid), ctypes.byref(h)))
        return _Borrowed(h, *self._queries[qid])

    def submit_update(self, qid: int, rel: int, keys, weights=None, unit_weights: bool = False) -> int:
        t = ctypes.c_uint64()
        _check(lib().cs_server_submit_update(self._s, int(qid), int(rel), ctypes.c_void_p(keys.data_ptr()),
                                             None if weights is None else ctypes.c_void_p(weights.data_ptr()),
                                             int(keys.shape[0]), UPDATE_UNIT_WEIGHTS if unit_weights else 0,
                                             ctypes.byref(t)))
        return t.value

    def submit_estimate(self, qid: int) -> int:
        t = ctypes.c_uint64()
        _check(lib().cs_server_submit_estimate(self._s, int(qid), ctypes.byref(t)))
        return t.value

    def poll(self, max_n: int = 4096):
        buf = (_Completion * max_n)()
        n = ctypes.c_int32()
        _check(lib().cs_server_poll(self._s, buf, max_n, ctypes.byref(n)))
        out = []
        for i in range(n.value):
            c = buf[i]
            d = dict(ticket=c.ticket, qid=c.qid, kind=c.kind, status=c.status, submit_us=c.submit_us,
                     start_us=c.start_us, done_us=c.done_us)
            if c.kind == 1:
                d["estimate"] = _estimate_dict(c.estimate, None)
            out.append(d)
        return out

    def drain(self):
        _check(lib().cs_server_drain(self._s))

    def stats(self) -> dict:
        st = _ServerStats()
        _check(lib().cs_server_stats(self._s, ctypes.byref(st)))
        return {f: getattr(st, f) for f, _ in _ServerStats._fields_ if f != "reserved"}


def _i128(lo: int, hi: int) -> int:
    v = (int(hi) & 0xFFFFFFFFFFFFFFFF) << 64 | (int(lo) & 0xFFFFFFFFFFFFFFFF)
    return v - (1 << 128) if v >= (1 << 127) else v


class AmsSketch:
    """The AMS multi-join sketch of Eq. 1 (the baseline): d x m int64 counters per
    relation, every tuple updating all of them."""

    def __init__(self, graph, m: int, d: int, seed: int):
        import torch
        if not torch.cuda.is_available():
            raise RuntimeError("csketch needs a HIP GPU; there is no CPU fallback")
        self.graph = graph
        self.m, self.d, self.seed = int(m), int(d), int(seed)
        h = ctypes.c_void_p()
        _check(lib().cs_ams_create(ctypes.byref(_graph_struct(graph)), self.m, self.d, self.seed, ctypes.byref(h)))
        self._h = h

    def close(self):
        if getattr(self, "_h", None):
            lib().cs_ams_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def update(self, rel: int, keys, weights=None, stream=None):
        n = int(keys.shape[0])
        _check(lib().cs_ams_update(self._h, int(rel), keys.data_ptr() if n else None,
                                   None if weights is None else weights.data_ptr(), n, _stream_ptr(stream)))

    def reset(self, stream=None):
        _check(lib().cs_ams_reset(self._h, _stream_ptr(stream)))

    def estimate(self, stream=None) -> dict:
        """Median X_t with the exact numerators S_t = m X_t of every repetition."""
        e = _AmsEstimate()
        lo = np.zeros(self.d, dtype=np.int64)
        hi = np.zeros(self.d, dtype=np.int64)
        ex = np.zeros(self.d, dtype=np.int32)
        _check(lib().cs_ams_estimate(self._h, _stream_ptr(stream), ctypes.byref(e), lo.ctypes.data, hi.ctypes.data,
                                     ex.ctypes.data))
        return {"value": e.value, "exact": bool(e.exact), "median_rep": e.median_rep,
                "numerator": _i128(e.num_lo, e.num_hi) if e.exact else None,
                "rep_numerators": [_i128(a, b) if c else None for a, b, c in zip(lo, hi, ex)]}

    def read_sketch(self, rel: int) -> np.ndarray:
        out = np.empty((self.d, self.m), dtype=np.int64)
        _check(lib().cs_ams_read(self._h, int(rel), out.ctypes.data))
        return out

    def coefficients(self) -> np.ndarray:
        n_edges = len(self.graph.edges)
        out = np.empty((self.d, self.m, n_edges, 4), dtype=np.uint64)
        _check(lib().cs_ams_coefficients(self._h, out.ctypes.data))
        return out


class AttrSketches:
    """One Count sketch per attribute of a query graph, with per-component hash functions
    (Sec. 3.4): one pass per relation updates all its attributes' sketches, and any two
    attributes of one component give their two-relation join estimate."""

    def __init__(self, graph, m: int, d: int, seed: int):
        import torch
        if not torch.cuda.is_available():
            raise RuntimeError("csketch needs a HIP GPU; there is no CPU fallback")
        self.graph = graph
        self.m, self.d, self.seed = int(m), int(d), int(seed)
        h = ctypes.c_void_p()
        _check(lib().cs_attr_create(ctypes.byref(_graph_struct(graph)), self.m, self.d, self.seed, ctypes.byref(h)))
        self._h = h

    def close(self):
        if getattr(self, "_h", None):
            lib().cs_attr_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def update(self, rel: int, keys, weights=None, stream=None, unit_weights: bool = False):
        n = int(keys.shape[0])
        _check(lib().cs_attr_update(self._h, int(rel), keys.data_ptr() if n else None,
                                    None if weights is None else weights.data_ptr(), n,
                                    UPDATE_UNIT_WEIGHTS if unit_weights else 0, _stream_ptr(stream)))

    def reset(self, stream=None):
        _check(lib().cs_attr_reset(self._h, _stream_ptr(stream)))

    def estimate_join(self, u: int, v: int, stream=None, reps: bool = False) -> dict:
        e = _Estimate()
        rp, arrs = _reps_struct(self.d) if reps else (None, None)
        _check(lib().cs_attr_estimate_join(self._h, int(u), int(v), _stream_ptr(stream), ctypes.byref(e),
                                           ctypes.byref(rp) if rp is not None else None))
        return _estimate_dict(e, arrs)

    def read_sketch(self, u: int) -> np.ndarray:
        out = np.empty((self.d, self.m), dtype=np.int64)
        _check(lib().cs_attr_read(self._h, int(u), out.ctypes.data))
        return out

    def coefficients(self):
        n_comp = _n_components(self.graph)
        sign = np.empty((self.d, n_comp, 4), dtype=np.uint64)
        bins = np.empty((self.d, n_comp, 2), dtype=np.uint64)
        _check(lib().cs_attr_coefficients(self._h, sign.ctypes.data, bins.ctypes.data))
        return sign, bins


class SubQueries:
    """Sketches of many sub-queries of one base query (Sec. 3.4): `sub_joins` lists each
    sub-query as a bit mask of the base graph's joins.  One pass per base relation
    updates every distinct sketch of that relation; sub-queries that join an attribute
    once share its sketch."""

    def __init__(self, graph, sub_joins, m: int, d: int, seed: int):
        import torch
        if not torch.cuda.is_available():
            raise RuntimeError("csketch needs a HIP GPU; there is no CPU fallback")
        self.graph = graph
        self.sub_joins = [int(x) for x in sub_joins]
        self.m, self.d, self.seed = int(m), int(d), int(seed)
        masks = np.array(self.sub_joins, dtype=np.uint32)
        h = ctypes.c_void_p()
        _check(lib().cs_subq_create(ctypes.byref(_graph_struct(graph)), masks.ctypes.data, len(self.sub_joins),
                                    self.m, self.d, self.seed, ctypes.byref(h)))
        self._h = h

    def close(self):
        if getattr(self, "_h", None):
            lib().cs_subq_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def update(self, rel: int, keys, weights=None, stream=None, unit_weights: bool = False):
        n = int(keys.shape[0])
        _check(lib().cs_subq_update(self._h, int(rel), keys.data_ptr() if n else None,
                                    None if weights is None else weights.data_ptr(), n,
                                    UPDATE_UNIT_WEIGHTS if unit_weights else 0, _stream_ptr(stream)))

    def reset(self, stream=None):
        _check(lib().cs_subq_reset(self._h, _stream_ptr(stream)))

    def estimate(self, q: int, stream=None, reps: bool = False) -> dict:
        e = _Estimate()
        rp, arrs = _reps_struct(self.d) if reps else (None, None)
        _check(lib().cs_subq_estimate(self._h, int(q), _stream_ptr(stream), ctypes.byref(e),
                                      ctypes.byref(rp) if rp is not None else None))
        return _estimate_dict(e, arrs)

    def estimate_all(self, stream=None) -> list:
        n = len(self.sub_joins)
        outs = (_Estimate * n)()
        _check(lib().cs_subq_estimate_all(self._h, _stream_ptr(stream), outs))
        return [_estimate_dict(outs[i], None) for i in range(n)]

    def layout(self):
        """(number of targets, target_of [n_sub][n_rel], -1 where a relation is absent)."""
        nt = ctypes.c_int32()
        tof = np.empty((len(self.sub_joins), self.graph.n_rel), dtype=np.int32)
        _check(lib().cs_subq_layout(self._h, ctypes.byref(nt), tof.ctypes.data))
        return nt.value, tof

    def read_target(self, target: int) -> np.ndarray:
        out = np.empty((self.d, self.m), dtype=np.int64)
        _check(lib().cs_subq_read(self._h, int(target), out.ctypes.data))
        return out

    def coefficients(self):
        n_comp = _n_components(self.graph)
        n_edge = len(self.graph.edges)
        cs = np.empty((self.d, n_comp, 4), dtype=np.uint64)
        bn = np.empty((self.d, n_comp, 2), dtype=np.uint64)
        es = np.empty((self.d, max(1, n_edge), 4), dtype=np.uint64)
        _check(lib().cs_subq_coefficients(self._h, cs.ctypes.data, bn.ctypes.data, es.ctypes.data))
        return cs, bn, es[:, :n_edge]


def _n_components(graph) -> int:
    """Connected components of the join graph's attributes."""
    parent = list(range(graph.n_attr))

    def find(a):
        while parent[a] != a:
            parent[a] = parent[parent[a]]
            a = parent[a]
        return a

    for u, v in graph.edges:
        parent[find(u)] = find(v)
    return len({find(u) for u in range(graph.n_attr)})


def import_sketch(blob: bytes, graph) -> "Sketch":
    """Re-create a handle from a cs_export blob (`graph` is kept on the Python side; the
    blob carries its own copy, which the library checks)."""
    h = ctypes.c_void_p()
    _check(lib().cs_import(blob, len(blob), ctypes.byref(h)))
    sk = Sketch.__new__(Sketch)
    sk.graph = graph
    sk.m = int.from_bytes(blob[12:16], "little")
    sk.d = int.from_bytes(blob[16:20], "little")
    sk.seed = int.from_bytes(blob[32:40], "little")
    sk._h = h
    return sk


ESTIMATE_BYTES = ctypes.sizeof(_Estimate)


def read_estimate(buf) -> dict:
    """A cs_estimate_t written by Sketch.estimate_async into a pinned host tensor (uint8,
    at least ESTIMATE_BYTES); call after the stream has passed the estimate."""
    e = _Estimate.from_buffer_copy(bytes(buf.numpy()[:ESTIMATE_BYTES]))
    return _estimate_dict(e, None)
