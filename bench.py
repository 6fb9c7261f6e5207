"""Benchmark of the sketch update + estimate hot path on one MI355X.

Workload (the metric's configuration): a 3-relation chain R1(A) - R2(A, B) - R3(B),
10^7 tuples per relation, uint32 keys Zipf(s = 1.1) over a domain of 10^6 per
attribute, m = 2^16 buckets, d = 9 repetitions, int64 counters, weights +1.  Keys are
generated on the GPU and resident in HBM before timing.

One step = the whole plain hot path over one batch: zero the counters, stream every
relation's tuples into its d x m sketches (one update launch per relation), then the
estimate (fp64 FFT spectral product-reduce, exactness step, median over d).

Printed: one JSON line.  `value` is tuple updates per second over whole steps.
`roofline` describes the dominant kernel (the hashing kernel of the two-column
relation), timed inside the timed steps with HIP events the library records around it
on the stream it runs on (events without the system-scope fence, so recording them
flushes no caches).  The per-relation update and estimate times come from a few
diagnostic steps after the timed ones.  `cpu_baseline` is the CPU oracle on a bounded
prefix of the same input, on this host.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "tuple updates/s into d×m count sketches + estimates/s; batched vs plain; p99 ms"
HBM_PEAK_GBS = 8000.0
# Horner-step peak (one v <- v * x + a mod 2^61 - 1 with a 32-bit key x): the chip
# issues 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz = 3.93e13 VALU lane-instructions/s, and
# the shortest step is 7 full-rate VALU instructions (2 v_mad_u64_u32, one move for the
# 64-bit addend, a 64-bit shift, an and, a 64-bit add of a and one 64-bit add folding
# the low 61 bits), so 5.62e12 steps/s.  A kernel made of nothing but independent
# steps reaches 5.32e12 steps/s on the chip.
ALU_STEP_PEAK = 256 * 4 * 16 * 2.4e9 / 7.0


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--n", type=int, default=10 ** 7, help="tuples per relation")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--cpu-tuples", type=int, default=1 << 22, help="oracle sample per relation")
    ap.add_argument("--strategy", type=int, default=0)
    ap.add_argument("--no-filtered", dest="filtered", action="store_false",
                    help="skip the filtered-ingestion section")
    ap.add_argument("--copy-probe", type=int, default=0,
                    help="only run a device copy of this many bytes (counter calibration) and exit")
    ap.add_argument("--batch-queries", type=int, default=4096,
                    help="batched section: chain/star queries (0 skips the section)")
    ap.add_argument("--serve-queries", type=int, default=256, help="serving section: live queries (0 skips)")
    ap.add_argument("--no-ams", dest="ams", action="store_false",
                    help="skip the AMS-baseline section (stream throughput at equal memory)")
    ap.add_argument("--anym", type=str, default="1000000,1048576",
                    help="bucket-count section: chain-3 steps at these m with d = 5 (empty skips)")
    ap.add_argument("--serve-seconds", type=float, default=3.0, help="serving section: seconds per load level")
    ap.add_argument("--serve-rates", type=str, default="250,1000,4000,16000",
                    help="serving section: offered update-batch arrival rates (batches/s)")
    return ap.parse_args()


TRAFFIC_PROFILE = os.path.join(ROOT, "profiles", "update_seg16_chain3_1e7_m65536_d9_traffic.md")
KERNEL_SOURCES = ["csk_update.hip", "csk_hash.h", "csk_counters16.h", "csk_internal.h"]


def kernel_source_digest() -> str:
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_2402_15953_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def measured_traffic(strategy: int):
    """HBM bytes per launch of the dominant kernel from the committed FETCH_SIZE and
    WRITE_SIZE counter summary (scaled by a copy kernel of known size), or None when the
    summary is missing, was taken for another strategy, or the kernel sources changed
    since the counters were taken."""
    if strategy != 0 or not os.path.exists(TRAFFIC_PROFILE):
        return None
    fields = {}
    with open(TRAFFIC_PROFILE) as fh:
        for line in fh:
            if ":" in line and line.startswith("- "):
                k, v = line[2:].split(":", 1)
                fields[k.strip()] = v.strip().strip("`")
    if fields.get("kernel_source_sha256") != kernel_source_digest():
        return None
    try:
        return float(fields["traffic_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def copy_probe(nbytes: int):
    """A plain device copy of known size (the scale for the FETCH_SIZE / WRITE_SIZE
    counters): five launches of dst.copy_(src) on nbytes."""
    import torch
    src = torch.ones(nbytes // 4, dtype=torch.int32, device="cuda")
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    for _ in range(5):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"copy_probe_bytes": src.numel() * 4, "launches": 5}), flush=True)


def horner_steps_per_tuple(graph, k, d):
    """d * sum over key columns (1 bin step + 3 steps per join at that attribute)."""
    steps = 0
    for u in graph.columns(k):
        joins = sum(1 for e in graph.edges if u in e)
        steps += 1 + 3 * joins
    return d * steps


def progress(msg: str):
    """One line per finished section on stderr (the JSON line stays alone on stdout)."""
    print("bench: " + msg, file=sys.stderr, flush=True)


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "the benchmark runs on one GPU; --gpus %d is not supported" % args.gpus}))
        print("bench.py runs on exactly one GPU (there is no multi-GPU path)", file=sys.stderr)
        sys.exit(2)
    if args.copy_probe > 0:
        copy_probe(args.copy_probe)
        return

    import numpy as np
    import torch

    import paper_2402_15953_amd as csk
    import workloads as W

    torch.cuda.set_device(0)
    dev = torch.device("cuda", 0)
    graph = W.chain(3)
    m, d, seed, n = 1 << 16, 9, 7, args.n
    s, D, config = 1.1, 10 ** 6, 2

    # ---- inputs resident in HBM (generated on the GPU, outside any timed region)
    keys = []
    for k in range(graph.n_rel):
        kk = W.relation_keys(graph, k, n, "zipf", config=config, s=s, D=D, device=dev)
        keys.append(kk.to(torch.int32).contiguous())
    torch.cuda.synchronize()

    stream = torch.cuda.Stream()
    t0 = time.perf_counter()
    sk = csk.Sketch(graph, m, d, seed)
    init_ms = (time.perf_counter() - t0) * 1e3

    n_rel = graph.n_rel
    ev = {k: [] for k in range(n_rel)}
    kev = {k: [] for k in range(n_rel)}   # around the hashing kernel alone (cs_update_timed)
    est_ev = []

    # timing events, made before the timed region (recording one costs no cache flush)
    n_diag = 3
    timers = iter([csk.Timer() for _ in range(args.steps * 2 * n_rel + n_diag * (n_rel + 2))])

    def step(mode):
        """mode 0: untimed; 1: timed step, the library records a pair around each hashing
        kernel; 2: diagnostic step (after the timed region), marks where each relation's
        update starts and around the estimate."""
        sk.reset(stream=stream)
        marks = []
        for k in range(n_rel):
            if mode == 1:
                ka, kb = next(timers), next(timers)
                sk.update(k, keys[k], None, stream=stream, strategy=args.strategy, timing=(ka, kb))
                kev[k].append((ka, kb))
                continue
            if mode == 2:
                a = next(timers)
                a.record(stream)
                marks.append(a)
            sk.update(k, keys[k], None, stream=stream, strategy=args.strategy)
        if mode == 2:
            a, b = next(timers), next(timers)
            a.record(stream)
            marks.append(a)
            for k in range(n_rel):
                ev[k].append((marks[k], marks[k + 1]))
        res = sk.estimate(stream=stream)
        if mode == 2:
            b.record(stream)
            est_ev.append((a, b))
        return res

    with torch.cuda.stream(stream):
        for _ in range(args.warmup):
            step(0)
        torch.cuda.synchronize()
        t_start = time.perf_counter()
        for _ in range(args.steps):
            res = step(1)
        torch.cuda.synchronize()
        elapsed = time.perf_counter() - t_start
        for _ in range(n_diag):
            step(2)
        torch.cuda.synchronize()

    # the same steps with the estimate published by the device (cs_estimate_async into
    # pinned memory, no host round trip per step); every step's result is checked after
    # the timed region against the synchronous estimate of the same counters
    pinned = [torch.zeros(csk.ESTIMATE_BYTES, dtype=torch.uint8, pin_memory=True) for _ in range(args.steps)]
    with torch.cuda.stream(stream):
        torch.cuda.synchronize()
        t_p = time.perf_counter()
        for i in range(args.steps):
            sk.reset(stream=stream)
            for k in range(n_rel):
                sk.update(k, keys[k], None, stream=stream, strategy=args.strategy)
            sk.estimate_async(pinned[i].data_ptr(), stream=stream)
        torch.cuda.synchronize()
        elapsed_p = time.perf_counter() - t_p
    pub = [csk.read_estimate(b) for b in pinned]
    pipelined = {"tuples_per_s": n * n_rel * args.steps / elapsed_p, "ms_per_step": elapsed_p * 1e3 / args.steps,
                 "identical_estimates": all(e["value"] == res["value"] and e["exact"] == res["exact"]
                                            and e["value_i64"] == res["value_i64"] for e in pub)}

    ms_per_step = elapsed * 1e3 / args.steps
    tuples_per_step = n * n_rel
    value = tuples_per_step * args.steps / elapsed
    upd_ms = {k: sum(a.elapsed_ms(b) for a, b in ev[k]) / len(ev[k]) for k in range(n_rel)}
    est_ms = sum(a.elapsed_ms(b) for a, b in est_ev) / len(est_ev)
    upd_total_ms = sum(upd_ms.values())

    kern_ms = {k: sum(a.elapsed_ms(b) for a, b in kev[k]) / len(kev[k]) for k in range(n_rel)}

    # dominant kernel: the slowest hashing kernel (one launch per relation and step)
    kdom = max(kern_ms, key=kern_ms.get)
    a_dom = len(graph.columns(kdom))
    bytes_dom = n * 4 * a_dom                       # uint32 keys, weights NULL
    steps_dom = n * horner_steps_per_tuple(graph, kdom, d)
    dur_s = kern_ms[kdom] / 1e3
    alu_achieved = steps_dom / dur_s
    hbm_achieved = bytes_dom / dur_s / 1e9
    traffic = measured_traffic(args.strategy)

    progress("plain step timed")
    out = {
        "metric": METRIC,
        "value": value,
        "unit": "tuple updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int64",
        "data": "synthetic",
        "config": {"workload": "chain3 R1(A)-R2(A,B)-R3(B), 1e7 tuples/relation, Zipf(1.1) over 1e6, "
                               "m=2^16, d=9, weights +1 (NULL)",
                   "relations": n_rel, "tuples_per_relation": n, "m": m, "d": d, "zipf_s": s, "domain": D,
                   "sketch_seed": seed, "data_seed_base": W.DATA_SEED_BASE},
        "roofline": {"bound": "alu", "achieved": alu_achieved / 1e12, "peak": ALU_STEP_PEAK / 1e12,
                     "unit": "T Horner-steps/s", "frac": alu_achieved / ALU_STEP_PEAK, "traffic": traffic,
                     "kernel": f"hashing kernel of relation {kdom}'s update ({a_dom} key columns)",
                     "kernel_ms": kern_ms[kdom], "algorithmic_bytes": bytes_dom,
                     "hbm_GBps": hbm_achieved, "hbm_frac": hbm_achieved / HBM_PEAK_GBS},
        "update_ms_per_relation": {str(k): v for k, v in upd_ms.items()},
        "hash_kernel_ms_per_relation": {str(k): v for k, v in kern_ms.items()},
        "update_tuples_per_s": tuples_per_step / (upd_total_ms / 1e3),
        "estimate_ms": est_ms,
        "estimates_per_s": 1e3 / est_ms,
        "init_ms": init_ms,
        "estimate": {"value": res["value"], "exact": res["exact"], "n_modular": res["n_modular"]},
        "pipelined_async_estimate": pipelined,
    }

    if args.filtered:
        out["filtered"] = bench_filtered(sk, keys, graph, dev, stream, args.steps)
        progress("filtered section done")
    sk.close()
    if args.anym:
        out["any_m"] = [bench_any_m(int(x), keys, graph, dev, stream, args.steps) for x in args.anym.split(",") if x]
        progress("any-m section done")
    if args.ams:
        out["ams_baseline"] = bench_ams(keys, graph, stream)
        progress("AMS section done")
    out["attr_sketches"] = bench_attr(keys, graph, stream, args.steps)
    progress("attribute-sketch section done")
    del keys
    torch.cuda.empty_cache()
    if args.batch_queries > 0:
        out["batched"] = bench_batched(args.batch_queries, dev, stream)
        progress("batched section done")
        torch.cuda.empty_cache()
    if args.serve_queries > 0:
        out["serving"] = bench_serving(args.serve_queries, dev, args.serve_seconds,
                                       [float(x) for x in args.serve_rates.split(",") if x])
        torch.cuda.empty_cache()
    if not args.no_cpu:
        keys_cpu = [W.relation_keys(graph, k, args.cpu_tuples, "zipf", config=config, s=s, D=D).to(torch.int32)
                    for k in range(graph.n_rel)]
        out["cpu_baseline"] = cpu_baseline(graph, keys_cpu, m, d, seed, args.cpu_tuples)
        progress("CPU baseline done")

    print(json.dumps(out), flush=True)


def bench_filtered(sk, keys, graph, dev, stream, steps):
    """The same chain-3 step with a filter at ingestion (Sec. 4.1): one uniform attribute
    column per relation over 0..99, kept when <= 24 (25% of the tuples pass)."""
    import torch

    import workloads as W
    n = keys[0].shape[0]
    attrs = [W.uniform_keys(n, 100, seed=W.data_seed(7, k, 9), device=dev).to(torch.int32).contiguous()
             for k in range(graph.n_rel)]
    preds = [(0, 0, 24)]
    kept = []

    def step():
        sk.reset(stream=stream)
        kept.clear()
        for k in range(graph.n_rel):
            kept.append(sk.update_filtered(k, keys[k], attrs[k], preds, stream=stream))
        return sk.estimate(stream=stream)

    with torch.cuda.stream(stream):
        step()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            res = step()
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / steps
    total = n * graph.n_rel
    return {"workload": "chain-3 step with one range predicate per relation at ingestion (25% kept)",
            "input_tuples_per_s": total / dt, "kept_fraction": sum(kept) / total, "ms_per_step": dt * 1e3,
            "estimate": res["value"]}


def bench_attr(keys, graph, stream, steps, m=1 << 16, d=9):
    """Per-attribute sketches of the chain-3 relations (Sec. 3.4 reuse): one pass per
    relation updates the sketches of all its attributes (R2's two columns in one pass),
    then the two pairwise joins are estimated from them."""
    import torch

    import paper_2402_15953_amd as csk
    ak = csk.AttrSketches(graph, m, d, 5)
    n = keys[0].shape[0]

    def step():
        ak.reset(stream=stream)
        for k in range(graph.n_rel):
            ak.update(k, keys[k], stream=stream)
        return [ak.estimate_join(u, v, stream=stream) for u, v in graph.edges]

    with torch.cuda.stream(stream):
        step()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            res = step()
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / steps
    ak.close()
    total = n * graph.n_rel
    return {"workload": f"chain-3 attribute sketches (4 attributes), 1e7 tuples/relation, m={m}, d={d}, "
                        "then both pairwise joins", "input_tuples_per_s": total / dt, "ms_per_step": dt * 1e3,
            "estimates": [r["value"] for r in res]}


def bench_ams(keys, graph, stream, d=5):
    """The stream-throughput comparison of Sec. 4 (its throughput table) on one GPU: the
    AMS multi-join sketch of Eq. 1 against the convolution sketch, chain-3, d = 5, at
    equal memory (counters plus hash coefficients) from 1 kB to 10 MB.  An AMS update
    touches all d x m counters, so its input is cut to about 4e10 hash steps a level."""
    import torch

    import paper_2402_15953_amd as csk
    r, E = graph.n_rel, len(graph.edges)
    Q = E  # chain: one component per join
    n_full = keys[0].shape[0]
    out = []

    def timed(fn, reps=3):
        best = float("inf")
        for _ in range(reps):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            fn()
            torch.cuda.synchronize()
            best = min(best, time.perf_counter() - t0)
        return best

    for mem in (1e3, 1e4, 1e5, 1e6, 1e7):
        m_ams = max(1, int(mem // (r * d * 8 + d * E * 4 * 8)))
        m_cs = max(2, int((mem - d * (4 * E + 2 * Q) * 8) // (r * d * 8)))
        n_ams = int(min(n_full, max(4096, 4e10 / (d * m_ams * 12))))
        ams = csk.AmsSketch(graph, m_ams, d, 3)
        cs = csk.Sketch(graph, m_cs, d, 3)
        with torch.cuda.stream(stream):
            def run_ams():
                ams.reset(stream=stream)
                for k in range(r):
                    ams.update(k, keys[k][:n_ams], stream=stream)

            def run_cs():
                cs.reset(stream=stream)
                for k in range(r):
                    cs.update(k, keys[k], None, stream=stream)

            run_ams()
            run_cs()
            t_ams = timed(run_ams)
            t_cs = timed(run_cs)
        out.append({"memory_bytes": mem, "ams_m": m_ams, "cs_m": m_cs, "ams_tuples": n_ams * r,
                    "ams_tuples_per_s": n_ams * r / t_ams, "cs_tuples_per_s": n_full * r / t_cs,
                    "ams_hash_steps_per_s": n_ams * d * m_ams * 3 * (2 * E) / t_ams})
        ams.close()
        cs.close()
    return {"workload": "chain-3, d=5, Zipf(1.1) keys, equal memory (counters + hash coefficients)",
            "levels": out}


def bench_any_m(m, keys, graph, dev, stream, steps, d=5):
    """The chain-3 step at the paper's sketch size (Sec. 4.1: m = 10^6 buckets, median of
    5), next to the nearest power of two: update throughput and estimate latency."""
    import torch

    import paper_2402_15953_amd as csk
    n = keys[0].shape[0]
    sk = csk.Sketch(graph, m, d, 11)
    tm = [csk.Timer() for _ in range(4 * steps)]
    upd, est = [], []

    def step(i):
        sk.reset(stream=stream)
        if i is not None:
            tm[4 * i].record(stream)
        for k in range(graph.n_rel):
            sk.update(k, keys[k], None, stream=stream)
        if i is not None:
            tm[4 * i + 1].record(stream)
            tm[4 * i + 2].record(stream)
        r = sk.estimate(stream=stream)
        if i is not None:
            tm[4 * i + 3].record(stream)
        return r

    with torch.cuda.stream(stream):
        step(None)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for i in range(steps):
            res = step(i)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / steps
    for i in range(steps):
        upd.append(tm[4 * i].elapsed_ms(tm[4 * i + 1]))
        est.append(tm[4 * i + 2].elapsed_ms(tm[4 * i + 3]))
    plan = {csk.PLAN_DOT: "dot", csk.PLAN_SPECTRAL: "spectral", csk.PLAN_GENERAL: "general"}[sk.info()["plan"]]
    sk.close()
    for t in tm:
        t.close()
    total = n * graph.n_rel
    return {"workload": f"chain-3 step, 1e7 tuples/relation, m={m}, d={d}", "m": m, "d": d, "plan": plan,
            "tuples_per_s": total / dt, "ms_per_step": dt * 1e3, "update_ms": sorted(upd)[len(upd) // 2],
            "estimate_ms": sorted(est)[len(est) // 2], "estimate": res["value"], "exact": res["exact"]}


def bench_batched(n_queries, dev, stream):
    """Uneven chain/star queries (2-6 relations, n log-uniform in [1e3, 1e6], m = 2^10..2^16,
    d in {5, 9}, Zipf(1.2) keys over 1e6): plain per-query calls vs one batched update
    (graph replay) and one batched estimate, on the same inputs."""
    import torch

    import paper_2402_15953_amd as csk
    import workloads as W

    specs = W.batched_queries(n_queries, seed=4)
    keys = []
    for qi, sp in enumerate(specs):
        keys.append([W.relation_keys(sp.graph, k, sp.n_per_rel[k], "zipf", config=4000 + qi, s=1.2, D=10 ** 6,
                                     device=dev).to(torch.int32).contiguous() for k in range(sp.graph.n_rel)])
    torch.cuda.synchronize()
    tuples = sum(sum(sp.n_per_rel) for sp in specs)
    sks = [csk.Sketch(sp.graph, sp.m, sp.d, sp.sketch_seed) for sp in specs]

    def plain_pass():
        t0 = time.perf_counter()
        for sk_, ks in zip(sks, keys):
            for k, kk in enumerate(ks):
                sk_.update(k, kk, stream=stream)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        ests = [sk_.estimate(stream=stream) for sk_ in sks]
        t2 = time.perf_counter()
        return t1 - t0, t2 - t1, ests

    def reset_all():
        for sk_ in sks:
            sk_.reset(stream=stream)
        torch.cuda.synchronize()

    plain_pass()                      # warm-up (kernel loading, scratch, workspaces)
    reset_all()
    t_up_plain, t_est_plain, est_plain = plain_pass()
    reset_all()
    b = csk.Batch()
    items = [(sk_, k, kk, None, False) for sk_, ks in zip(sks, keys) for k, kk in enumerate(ks)]
    t0 = time.perf_counter()
    b.capture(items, stream=stream)   # plans the work list (host) and captures the launch
    t_plan = time.perf_counter() - t0
    b.replay(stream=stream)
    torch.cuda.synchronize()
    b.estimate(sks, stream=stream)    # warm-up of the batched estimate workspace
    reset_all()
    t0 = time.perf_counter()
    b.replay(stream=stream)
    torch.cuda.synchronize()
    t_up_batch = time.perf_counter() - t0
    t0 = time.perf_counter()
    est_batch = b.estimate(sks, stream=stream)
    t_est_batch = time.perf_counter() - t0
    stats = b.stats()
    b.close()
    identical = est_batch == est_plain
    for sk_ in sks:
        sk_.close()
    return {"workload": f"{n_queries} chain/star queries, 2-6 relations, n log-uniform [1e3,1e6], "
                        "m=2^10..2^16, d in {5,9}, Zipf(1.2) over 1e6, weights +1",
            "tuples": tuples,
            "plain_update_tuples_per_s": tuples / t_up_plain, "batched_update_tuples_per_s": tuples / t_up_batch,
            "plain_estimates_per_s": n_queries / t_est_plain, "batched_estimates_per_s": n_queries / t_est_batch,
            "update_speedup": t_up_plain / t_up_batch, "estimate_speedup": t_est_plain / t_est_batch,
            "batched_plan_s": t_plan, "tasks": stats, "identical_estimates": identical}


def bench_serving(n_queries, dev, seconds, rates):
    """Live chain/star queries (m = 2^14..2^18, d = 9), Poisson arrivals of turnstile update
    batches (2^U[10,18] tuples, 10% deletes of earlier batches, weights +-1) and estimate
    requests at 1 estimate per 4 update batches; latency per request = completion - arrival."""
    import random

    import numpy as np
    import torch

    import paper_2402_15953_amd as csk
    import workloads as W

    specs = W.batched_queries(n_queries, seed=5, m_log2=(14, 18), d_choices=(9,), n_range=(1, 2))
    pool = 1 << 18
    pools = [[W.relation_keys(sp.graph, k, pool, "zipf", config=5000 + qi, s=1.1, D=10 ** 6,
                              device=dev).to(torch.int32).contiguous() for k in range(sp.graph.n_rel)]
             for qi, sp in enumerate(specs)]
    ones = torch.ones(pool, dtype=torch.int64, device=dev)
    minus = -ones
    torch.cuda.synchronize()
    srv = csk.Server(n_streams=3, max_batch_items=1024)
    qids = [srv.add_query(sp.graph, sp.m, sp.d, sp.sketch_seed) for sp in specs]
    # warm-up: one small update and one estimate per query (kernel loading, twiddle
    # tables, estimate workspace), then reset to empty sketches
    for qi, sp in enumerate(specs):
        srv.submit_update(qids[qi], 0, pools[qi][0][:1024], ones[:1024], unit_weights=True)
        srv.submit_estimate(qids[qi])
        srv.submit_update(qids[qi], 0, pools[qi][0][:1024], minus[:1024], unit_weights=True)
    srv.drain()
    srv.poll(1 << 20)
    levels = []
    rng = random.Random(9)
    inserted = {}
    # an unrecorded first window at the lowest rate (1 s) takes the one-time costs that
    # real-sized sketches bring (first modular estimates, workspace growth) out of the
    # measured levels
    for li, rate in enumerate([rates[0]] + list(rates)):
        window = 1.0 if li == 0 else seconds
        plan = []
        t = 0.0
        total_rate = rate * 1.25          # update batches + estimates (1:4)
        while t < window:
            t += rng.expovariate(total_rate)
            q = rng.randrange(n_queries)
            if rng.random() < 0.2:
                plan.append((t, "E", q, 0, 0, 0, 0))
                continue
            k = rng.randrange(specs[q].graph.n_rel)
            prev = inserted.get((q, k), [])
            if prev and rng.random() < 0.1:
                off, ln = prev.pop(rng.randrange(len(prev)))
                plan.append((t, "U", q, k, off, ln, -1))
            else:
                ln = 1 << rng.randint(10, 18)
                off = rng.randrange(0, pool - ln + 1)
                inserted.setdefault((q, k), []).append((off, ln))
                plan.append((t, "U", q, k, off, ln, 1))
        srv.drain()
        srv.poll(1 << 20)
        t0 = time.perf_counter()
        tuples = 0
        busy = 0
        for (ta, kind, q, k, off, ln, sign) in plan:
            while time.perf_counter() - t0 < ta:
                pass
            try:
                if kind == "U":
                    srv.submit_update(qids[q], k, pools[q][k][off:off + ln],
                                      (ones if sign > 0 else minus)[off:off + ln], unit_weights=True)
                    tuples += ln
                else:
                    srv.submit_estimate(qids[q])
            except csk.CsError:
                busy += 1
        srv.drain()
        wall = time.perf_counter() - t0
        comps = srv.poll(1 << 20)
        lat_u = np.array([c["done_us"] - c["submit_us"] for c in comps if c["kind"] == 0]) / 1e3
        lat_e = np.array([c["done_us"] - c["submit_us"] for c in comps if c["kind"] == 1]) / 1e3
        n_e = int(len(lat_e))

        def pct(a, p):
            return float(np.percentile(a, p)) if len(a) else None

        progress("serving window at %g batches/s done%s" % (rate, " (warm-up)" if li == 0 else ""))
        if li == 0:
            continue
        levels.append({"offered_update_batches_per_s": rate, "offered_estimates_per_s": rate / 4,
                       "seconds": wall, "tuples_per_s": tuples / wall, "estimates_per_s": n_e / wall,
                       "update_p50_ms": pct(lat_u, 50), "update_p99_ms": pct(lat_u, 99),
                       "estimate_p50_ms": pct(lat_e, 50), "estimate_p99_ms": pct(lat_e, 99),
                       "requests": len(comps), "refused": busy})
    st = srv.stats()
    srv.close()
    return {"workload": f"{n_queries} live chain/star queries, m=2^14..2^18, d=9, Zipf(1.1) over 1e6, "
                        "update batches 2^U[10,18] tuples, 10% deletes, estimate:update = 1:4, Poisson arrivals",
            "resident_counter_bytes": int(st["used_bytes"]), "levels": levels,
            "update_launches": int(st["update_launches"]), "estimate_batches": int(st["estimate_batches"])}


def cpu_baseline(graph, keys, m, d, seed, n_sample):
    """The oracle (plain C sketch loop + exact NTT estimate) on the first n_sample
    tuples of every relation: tuples per second of the same step on this host."""
    import numpy as np

    import oracle

    info = oracle.analyze(graph)
    co = oracle.draw_coefficients(seed, d, len(info.edges), info.n_comp)
    host = [k[:n_sample].cpu().numpy().view(np.uint32).reshape(n_sample, -1) for k in keys]
    t0 = time.perf_counter()
    sks = [oracle.create_sketch(info, k, host[k], None, m, co) for k in range(graph.n_rel)]
    t1 = time.perf_counter()
    oracle.estimate(info, sks, m, method="ntt")
    t2 = time.perf_counter()
    tuples = n_sample * graph.n_rel
    return {"value": tuples / (t2 - t0), "unit": "tuple updates/s", "cores": 1, "kind": "oracle",
            "sample": f"first {n_sample} tuples of each of the {graph.n_rel} relations "
                      f"(sketch {t1 - t0:.2f} s + exact estimate {t2 - t1:.2f} s)",
            "update_only_tuples_per_s": tuples / (t1 - t0), "estimate_s": t2 - t1}


if __name__ == "__main__":
    main()
