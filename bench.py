"""Benchmark of the sketch update + estimate hot path on one MI355X.

Headline workload (the largest single-GPU configuration of the metric): a 5-relation
chain R1(A) - R2(A, B) - R3(B, C) - R4(C, D) - R5(D), each relation streamed as 96 calls
of 2^20 tuples (100,663,296 tuples per relation), uint32 keys Zipf(s) over a domain of
10^7 per attribute for s in {0.5, 1.0, 1.5}, m = 2^18 buckets, d = 15 repetitions,
int64 counters, weights +1.  Keys are generated on the GPU and resident in HBM (9.7 GB)
before timing.

One step = the whole plain hot path over one batch: for each of the three exponents,
zero that query's counters, stream every relation's tuples into its d x m sketches
(480 update calls), then the estimate (fp64 FFT spectral product-reduce, exactness
step, median over d).

Printed: one JSON line.  `value` is tuple updates per second over whole steps.
`roofline` describes the dominant kernel (the hashing pass of a two-column relation's
update), timed inside the timed steps with HIP events the library records around it on
the stream it runs on (events without the system-scope fence, so recording them flushes
no caches), against the Horner-step peak; the same run measures that peak and the HBM
stream-read rate with the library's probe kernels (`k0`).  Per-relation update and
estimate times come from a diagnostic step after the timed ones.  Sections: the
3-relation chain (10^7 tuples per relation, m = 2^16, d = 9), the single join (10^5
tuples, m = 1024, d = 5), filtered ingestion, the paper's m = 10^6, the AMS baseline,
per-attribute sketches, 4096 batched queries, the serving loop.  `cpu_baseline` is the
CPU oracle on a bounded prefix of the headline input, on this host's cores.
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
# the low 61 bits), so 5.62e12 steps/s.  The probe kernel of independent steps
# (cs_k0_horner) measures what the chip sustains in the same run.
ALU_STEP_PEAK = 256 * 4 * 16 * 2.4e9 / 7.0
SECTIONS = ("chain5", "chain3", "single", "k0", "filtered", "anym", "ams", "attr", "subq", "batched", "serving",
            "cpu")


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--sections", type=str, default=",".join(SECTIONS),
                    help="comma-separated subset of " + ",".join(SECTIONS))
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--cpu-slices", type=int, default=8,
                    help="CPU baseline: 2^20-tuple slices per relation for the threaded oracle")
    ap.add_argument("--strategy", type=int, default=0)
    ap.add_argument("--chain5-calls", type=int, default=96,
                    help="headline: update calls of 2^20 tuples per relation (fewer only for profiling)")
    ap.add_argument("--copy-probe", type=int, default=0,
                    help="only run a device copy of this many bytes (counter calibration) and exit")
    ap.add_argument("--batch-queries", type=int, default=4096,
                    help="batched section: chain/star queries (0 skips the section)")
    ap.add_argument("--serve-queries", type=int, default=256, help="serving section: live queries (0 skips)")
    ap.add_argument("--anym", type=str, default="1000000,1048576",
                    help="bucket-count section: chain-3 steps at these m with d = 5 (empty skips)")
    ap.add_argument("--serve-seconds", type=float, default=3.0, help="serving section: seconds per load level")
    ap.add_argument("--serve-rates", type=str, default="250,1000,4000,16000",
                    help="serving section: offered update-batch arrival rates (batches/s)")
    return ap.parse_args()


TRAFFIC_PROFILES = {
    # dominant kernel -> committed FETCH_SIZE / WRITE_SIZE summary
    "chain5": os.path.join(ROOT, "profiles", "part_hash_chain5_2p20_m262144_d15_traffic.md"),
    "chain3": os.path.join(ROOT, "profiles", "update_seg16_chain3_1e7_m65536_d9_traffic.md"),
}
KERNEL_SOURCES = ["csk_update.hip", "csk_hash.h", "csk_counters16.h", "csk_internal.h"]


def kernel_source_digest() -> str:
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_2402_15953_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def launch_ms(pairs):
    """Duration of a kernel from its (start, stop) event pairs: the median launch (a
    sampled pair caught in a rare stall, once seen at 15x the others, would move a mean
    by tens of percent), with the mean and the extremes kept beside it."""
    v = sorted(a_.elapsed_ms(b_) for a_, b_ in pairs)
    n = len(v)
    med = v[n // 2] if n % 2 else 0.5 * (v[n // 2 - 1] + v[n // 2])
    return med, {"launches": n, "median_ms": med, "mean_ms": sum(v) / n, "min_ms": v[0], "max_ms": v[-1]}


def measured_traffic(which: str, strategy: int):
    """HBM bytes per launch of the dominant kernel from the committed FETCH_SIZE and
    WRITE_SIZE counter summary (scaled by a copy kernel of known size), or None when the
    summary is missing, was taken for another strategy, or the kernel sources changed
    since the counters were taken."""
    path = TRAFFIC_PROFILES.get(which)
    if strategy != 0 or not path or not os.path.exists(path):
        return None
    fields = {}
    with open(path) as fh:
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


def median(xs):
    s = sorted(xs)
    return s[len(s) // 2]


def bench_chain5(args, dev, stream):
    """The headline: 5-chain, 96 calls of 2^20 tuples per relation, m = 2^18, d = 15, for
    each of Zipf s in {0.5, 1.0, 1.5} (one query handle per exponent)."""
    import torch

    import paper_2402_15953_amd as csk
    import workloads as W

    graph = W.chain(5)
    m, d, seed, D, config = 1 << 18, 15, 8, 10 ** 7, 3
    n_call, calls = 1 << 20, args.chain5_calls
    n = n_call * calls
    exps = (0.5, 1.0, 1.5)
    r = graph.n_rel
    keys = {}
    for sx in exps:
        keys[sx] = [W.relation_keys(graph, k, n, "zipf", config=config, s=sx, D=D, device=dev)
                    .to(torch.int32).contiguous() for k in range(r)]
    torch.cuda.synchronize()
    progress("chain5 keys resident (%.1f GB)" % (sum(x.numel() * 4 for v in keys.values() for x in v) / 1e9))
    t0 = time.perf_counter()
    sks = {sx: csk.Sketch(graph, m, d, seed) for sx in exps}
    init_ms = (time.perf_counter() - t0) * 1e3 / len(exps)
    sampled_calls = tuple(sorted(set(min(calls - 1, c) for c in (0, 31, 63, 95))))
    kev = {k: [] for k in range(r)}
    n_timers = args.steps * len(exps) * r * len(sampled_calls) * 2 + len(exps) * (r + 2) + 8
    timers = iter([csk.Timer() for _ in range(n_timers)])
    diag = {}

    def step(mode):
        """mode 0: untimed; 1: timed, the library records a pair around the hashing
        kernel of sampled calls; 2: diagnostic, marks at each relation's start and
        around the estimate."""
        out = {}
        for sx in exps:
            sk = sks[sx]
            ks = keys[sx]
            sk.reset(stream=stream)
            marks = []
            for k in range(r):
                if mode == 2:
                    a_ = next(timers)
                    a_.record(stream)
                    marks.append(a_)
                for c in range(calls):
                    part = ks[k][c * n_call:(c + 1) * n_call]
                    if mode == 1 and c in sampled_calls:
                        ka, kb = next(timers), next(timers)
                        sk.update(k, part, None, stream=stream, strategy=args.strategy, timing=(ka, kb))
                        kev[k].append((ka, kb))
                    else:
                        sk.update(k, part, None, stream=stream, strategy=args.strategy)
            if mode == 2:
                a_, b_ = next(timers), next(timers)
                a_.record(stream)
                marks.append(a_)
            out[sx] = sk.estimate(stream=stream)
            if mode == 2:
                b_.record(stream)
                diag[sx] = (marks, b_)
        return out

    with torch.cuda.stream(stream):
        for _ in range(args.warmup):
            step(0)
        torch.cuda.synchronize()
        t_start = time.perf_counter()
        for _ in range(args.steps):
            res = step(1)
        torch.cuda.synchronize()
        elapsed = time.perf_counter() - t_start
        step(2)
        torch.cuda.synchronize()

    tuples_per_step = n * r * len(exps)
    value = tuples_per_step * args.steps / elapsed
    kern_stat = {k: launch_ms(kev[k]) for k in range(r)}
    kern_ms = {k: v[0] for k, v in kern_stat.items()}
    upd_ms = {}   # per exponent and relation: the 96 calls, both passes
    est_ms = {}
    for sx in exps:
        marks, b_ = diag[sx]
        upd_ms[str(sx)] = {str(k): marks[k].elapsed_ms(marks[k + 1]) for k in range(r)}
        est_ms[str(sx)] = marks[r].elapsed_ms(b_)
    kdom = max(kern_ms, key=kern_ms.get)
    a_dom = len(graph.columns(kdom))
    steps_dom = n_call * horner_steps_per_tuple(graph, kdom, d)
    bytes_dom = n_call * 4 * a_dom
    dur_s = kern_ms[kdom] / 1e3
    alu_achieved = steps_dom / dur_s
    hbm_achieved = bytes_dom / dur_s / 1e9
    steps_all = sum(n * horner_steps_per_tuple(graph, k, d) for k in range(r))
    upd_all_ms = {sx: sum(v.values()) for sx, v in upd_ms.items()}
    est_bytes = r * d * m * 8
    est_mean = sum(est_ms.values()) / len(est_ms)
    out = {
        "value": value, "ms_per_step": elapsed * 1e3 / args.steps, "tuples_per_step": tuples_per_step,
        "config": {"workload": "chain5 R1(A)-R2(A,B)-R3(B,C)-R4(C,D)-R5(D), 96 update calls of 2^20 tuples per "
                               "relation, Zipf s in {0.5, 1.0, 1.5} over 1e7, m=2^18, d=15, weights +1 (NULL); "
                               "one step = all three exponents' streams and estimates",
                   "relations": r, "tuples_per_relation": n, "calls_per_relation": calls, "tuples_per_call": n_call,
                   "m": m, "d": d, "zipf_s": list(exps), "domain": D, "sketch_seed": seed,
                   "data_seed_base": W.DATA_SEED_BASE},
        "roofline": {"bound": "alu", "achieved": alu_achieved / 1e12, "peak": ALU_STEP_PEAK / 1e12,
                     "unit": "T Horner-steps/s", "frac": alu_achieved / ALU_STEP_PEAK,
                     "traffic": measured_traffic("chain5", args.strategy),
                     "kernel": f"hashing pass (k_part_hash) of relation {kdom}'s update ({a_dom} key columns), "
                               f"one launch per 2^20-tuple call",
                     "kernel_ms": kern_ms[kdom], "kernel_launches": kern_stat[kdom][1],
                     "algorithmic_steps": steps_dom, "algorithmic_bytes": bytes_dom,
                     "hbm_GBps": hbm_achieved, "hbm_frac": hbm_achieved / HBM_PEAK_GBS},
        "hash_kernel_ms_per_call": {str(k): v for k, v in kern_ms.items()},
        "update_ms_per_relation": upd_ms,
        "update_step_frac": {sx: steps_all / (v / 1e3) / ALU_STEP_PEAK for sx, v in upd_all_ms.items()},
        "update_tuples_per_s": {sx: n * r / (v / 1e3) for sx, v in upd_all_ms.items()},
        "estimate_ms": est_ms,
        "estimates_per_s": 1e3 / est_mean,
        "estimate_roofline": {"bound": "hbm", "algorithmic_bytes": est_bytes,
                              "achieved_GBps": est_bytes / (est_mean / 1e3) / 1e9,
                              "frac": est_bytes / (est_mean / 1e3) / 1e9 / HBM_PEAK_GBS},
        "init_ms": init_ms,
        "estimates": {str(sx): {"value": v["value"], "exact": v["exact"], "n_modular": v["n_modular"]}
                      for sx, v in res.items()},
    }
    for sk in sks.values():
        sk.close()
    host0 = [keys[1.0][k][:n_call * args.cpu_slices].cpu() for k in range(r)]
    probe_buf = keys[1.0][1]
    return out, host0, probe_buf, keys


def bench_chain3(args, dev, stream):
    """The 3-relation chain: 10^7 tuples per relation, Zipf(1.1) over 10^6, m = 2^16, d = 9."""
    import torch

    import paper_2402_15953_amd as csk
    import workloads as W

    graph = W.chain(3)
    m, d, seed, n = 1 << 16, 9, 7, 10 ** 7
    s, D, config = 1.1, 10 ** 6, 2
    keys = [W.relation_keys(graph, k, n, "zipf", config=config, s=s, D=D, device=dev).to(torch.int32).contiguous()
            for k in range(graph.n_rel)]
    torch.cuda.synchronize()
    sk = csk.Sketch(graph, m, d, seed)
    n_rel = graph.n_rel
    ev = {k: [] for k in range(n_rel)}
    kev = {k: [] for k in range(n_rel)}
    est_ev = []
    n_diag = 3
    timers = iter([csk.Timer() for _ in range(args.steps * 2 * n_rel + n_diag * (n_rel + 2))])

    def step(mode):
        sk.reset(stream=stream)
        marks = []
        for k in range(n_rel):
            if mode == 1:
                ka, kb = next(timers), next(timers)
                sk.update(k, keys[k], None, stream=stream, strategy=args.strategy, timing=(ka, kb))
                kev[k].append((ka, kb))
                continue
            if mode == 2:
                a_ = next(timers)
                a_.record(stream)
                marks.append(a_)
            sk.update(k, keys[k], None, stream=stream, strategy=args.strategy)
        if mode == 2:
            a_, b_ = next(timers), next(timers)
            a_.record(stream)
            marks.append(a_)
            for k in range(n_rel):
                ev[k].append((marks[k], marks[k + 1]))
        res_ = sk.estimate(stream=stream)
        if mode == 2:
            b_.record(stream)
            est_ev.append((a_, b_))
        return res_

    with torch.cuda.stream(stream):
        for _ in range(max(1, args.warmup)):
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
    # pinned memory, no host round trip per step), checked against the synchronous one
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
    kern_stat = {k: launch_ms(kev[k]) for k in range(n_rel)}
    kern_ms = {k: v[0] for k, v in kern_stat.items()}
    upd_ms = {k: sum(a_.elapsed_ms(b_) for a_, b_ in ev[k]) / len(ev[k]) for k in range(n_rel)}
    est_ms = sum(a_.elapsed_ms(b_) for a_, b_ in est_ev) / len(est_ev)
    kdom = max(kern_ms, key=kern_ms.get)
    a_dom = len(graph.columns(kdom))
    steps_dom = n * horner_steps_per_tuple(graph, kdom, d)
    dur_s = kern_ms[kdom] / 1e3
    est_bytes = n_rel * d * m * 8
    sk.close()
    tuples_per_step = n * n_rel
    return {
        "workload": "chain3 R1(A)-R2(A,B)-R3(B), 1e7 tuples/relation (one update call each), Zipf(1.1) over 1e6, "
                    "m=2^16, d=9, weights +1 (NULL)",
        "tuples_per_s": tuples_per_step * args.steps / elapsed, "ms_per_step": elapsed * 1e3 / args.steps,
        "roofline": {"bound": "alu", "achieved": steps_dom / dur_s / 1e12, "peak": ALU_STEP_PEAK / 1e12,
                     "unit": "T Horner-steps/s", "frac": steps_dom / dur_s / ALU_STEP_PEAK,
                     "traffic": measured_traffic("chain3", args.strategy),
                     "kernel": f"hashing kernel of relation {kdom}'s update ({a_dom} key columns)",
                     "kernel_ms": kern_ms[kdom], "kernel_launches": kern_stat[kdom][1],
                     "algorithmic_bytes": n * 4 * a_dom,
                     "hbm_frac": n * 4 * a_dom / dur_s / 1e9 / HBM_PEAK_GBS},
        "hash_kernel_ms_per_relation": {str(k): v for k, v in kern_ms.items()},
        "update_ms_per_relation": {str(k): v for k, v in upd_ms.items()},
        "update_tuples_per_s": tuples_per_step / (sum(upd_ms.values()) / 1e3),
        "estimate_ms": est_ms, "estimates_per_s": 1e3 / est_ms,
        "estimate_roofline": {"bound": "hbm", "algorithmic_bytes": est_bytes,
                              "achieved_GBps": est_bytes / (est_ms / 1e3) / 1e9,
                              "frac": est_bytes / (est_ms / 1e3) / 1e9 / HBM_PEAK_GBS},
        "estimate": {"value": res["value"], "exact": res["exact"], "n_modular": res["n_modular"]},
        "pipelined_async_estimate": {
            "tuples_per_s": tuples_per_step * args.steps / elapsed_p, "ms_per_step": elapsed_p * 1e3 / args.steps,
            "identical_estimates": all(e["value"] == res["value"] and e["exact"] == res["exact"]
                                       and e["value_i64"] == res["value_i64"] for e in pub)},
    }, keys


def bench_single(args, dev, stream):
    """The single equi-join R1(A) - R2(A): 10^5 tuples each, keys uniform on [0, 10^4),
    m = 1024, d = 5 (the inner-product plan), against the exact join size."""
    import numpy as np
    import torch

    import paper_2402_15953_amd as csk
    import workloads as W

    graph = W.single_join()
    n, m, d, seed = 10 ** 5, 1024, 5, 7
    keys = [W.relation_keys(graph, k, n, "uniform", config=1, D=10 ** 4, device=dev).to(torch.int32).contiguous()
            for k in range(2)]
    torch.cuda.synchronize()
    sk = csk.Sketch(graph, m, d, seed)
    reps = 200

    def step():
        sk.reset(stream=stream)
        for k in range(2):
            sk.update(k, keys[k], None, stream=stream)
        return sk.estimate(stream=stream)

    with torch.cuda.stream(stream):
        step()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            res = step()
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / reps
        t1 = time.perf_counter()
        for _ in range(reps):
            sk.estimate(stream=stream)
        de = (time.perf_counter() - t1) / reps
    h = [np.bincount(keys[k].cpu().numpy().ravel(), minlength=10 ** 4) for k in range(2)]
    exact = int(np.dot(h[0].astype(np.int64), h[1].astype(np.int64)))
    sk.close()
    return {"workload": "single join R1(A)-R2(A), 1e5 tuples each, uniform keys on [0,1e4), m=1024, d=5, weights +1",
            "tuples_per_s": 2 * n / dt, "ms_per_step": dt * 1e3, "estimates_per_s": 1 / de,
            "estimate": res["value"], "exact": res["exact"], "true_join_size": exact,
            "relative_error": abs(res["value"] - exact) / exact}


def bench_k0(probe_buf):
    """The two machine-balance rates measured by the library's probe kernels."""
    import paper_2402_15953_amd as csk
    steps = max(csk.k0_horner(1 << 14) for _ in range(3))
    read = max(csk.k0_stream_read(probe_buf, 5) for _ in range(2))
    return {"horner_steps_per_s": steps, "horner_frac_of_peak": steps / ALU_STEP_PEAK,
            "stream_read_GBps": read / 1e9, "stream_read_frac_of_peak": read / 1e9 / HBM_PEAK_GBS,
            "stream_read_bytes": probe_buf.numel() * probe_buf.element_size()}


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "the benchmark runs on one GPU; --gpus %d is not supported" % args.gpus}))
        print("bench.py runs on exactly one GPU (there is no multi-GPU path)", file=sys.stderr)
        sys.exit(2)
    if args.copy_probe > 0:
        copy_probe(args.copy_probe)
        return
    sections = set(x for x in args.sections.split(",") if x)
    if args.no_cpu:
        sections.discard("cpu")

    import torch

    torch.cuda.set_device(0)
    dev = torch.device("cuda", 0)
    stream = torch.cuda.Stream()
    out = {"metric": METRIC, "value": None, "unit": "tuple updates/s", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "ms_per_step": None, "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": "int64", "data": "synthetic"}
    host0 = None
    if "chain5" in sections:
        head, host0, probe_buf, keys5 = bench_chain5(args, dev, stream)
        out["value"] = head.pop("value")
        out["ms_per_step"] = head.pop("ms_per_step")
        out["config"] = head.pop("config")
        out["roofline"] = head.pop("roofline")
        out.update(head)
        progress("chain5 headline timed")
        if "k0" in sections:
            out["k0"] = bench_k0(probe_buf)
            out["roofline"]["frac_of_k0"] = out["roofline"]["achieved"] * 1e12 / out["k0"]["horner_steps_per_s"]
            progress("k0 probes done")
        del probe_buf, keys5
        torch.cuda.empty_cache()
    keys3 = None
    if "chain3" in sections:
        out["chain3"], keys3 = bench_chain3(args, dev, stream)
        progress("chain3 section done")
    if "single" in sections:
        out["single_join"] = bench_single(args, dev, stream)
        progress("single-join section done")
    if keys3 is not None:
        import workloads as W
        g3 = W.chain(3)
        if "filtered" in sections:
            out["filtered"] = bench_filtered(keys3, g3, dev, stream, args.steps)
            progress("filtered section done")
        if "anym" in sections and args.anym:
            out["any_m"] = [bench_any_m(int(x), keys3, g3, dev, stream, args.steps) for x in args.anym.split(",") if x]
            progress("any-m section done")
        if "ams" in sections:
            out["ams_baseline"] = bench_ams(keys3, g3, stream)
            progress("AMS section done")
        if "attr" in sections:
            out["attr_sketches"] = bench_attr(keys3, g3, stream, args.steps)
            progress("attribute-sketch section done")
        del keys3
        torch.cuda.empty_cache()
    if "subq" in sections:
        out["subqueries"] = bench_subq(dev, stream, args.steps)
        progress("sub-query section done")
        torch.cuda.empty_cache()
    if "batched" in sections and args.batch_queries > 0:
        out["batched"] = bench_batched(args.batch_queries, dev, stream)
        progress("batched section done")
        torch.cuda.empty_cache()
    if "serving" in sections and args.serve_queries > 0:
        out["serving"] = bench_serving(args.serve_queries, dev, args.serve_seconds,
                                       [float(x) for x in args.serve_rates.split(",") if x], stream)
        torch.cuda.empty_cache()
    if "cpu" in sections and host0 is not None:
        out["cpu_baseline"] = cpu_baseline(host0)
        progress("CPU baseline done")
    print(json.dumps(out), flush=True)


def bench_filtered(keys, graph, dev, stream, steps, m=1 << 16, d=9):
    """The chain-3 step with a filter at ingestion (Sec. 4.1): one uniform attribute column
    per relation over 0..99, kept when <= 24 (25% of the tuples pass), beside the same
    step unfiltered."""
    import torch

    import paper_2402_15953_amd as csk
    import workloads as W
    n = keys[0].shape[0]
    attrs = [W.uniform_keys(n, 100, seed=W.data_seed(7, k, 9), device=dev).to(torch.int32).contiguous()
             for k in range(graph.n_rel)]
    preds = [(0, 0, 24)]
    sk = csk.Sketch(graph, m, d, 7)

    def step(filtered):
        sk.reset(stream=stream)
        for k in range(graph.n_rel):
            if filtered:
                sk.update_filtered(k, keys[k], attrs[k], preds, stream=stream, count=False)
            else:
                sk.update(k, keys[k], None, stream=stream)
        return sk.estimate(stream=stream)

    times, upd = {}, {}
    with torch.cuda.stream(stream):
        for filtered in (False, True):
            step(filtered)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(steps):
                res = step(filtered)
            torch.cuda.synchronize()
            times[filtered] = (time.perf_counter() - t0) / steps
            # the updates alone (three relations), between two timing events
            ta, tb = csk.Timer(), csk.Timer()
            sk.reset(stream=stream)
            ta.record(stream)
            for k in range(graph.n_rel):
                if filtered:
                    sk.update_filtered(k, keys[k], attrs[k], preds, stream=stream, count=False)
                else:
                    sk.update(k, keys[k], None, stream=stream)
            tb.record(stream)
            torch.cuda.synchronize()
            upd[filtered] = ta.elapsed_ms(tb)
    kept = [int(((a >= 0) & (a <= 24)).sum().item()) for a in attrs]
    sk.close()
    total = n * graph.n_rel
    return {"workload": "chain-3 step with one range predicate per relation at ingestion (25% kept)",
            "input_tuples_per_s": total / times[True], "kept_fraction": sum(kept) / total,
            "ms_per_step": times[True] * 1e3, "unfiltered_ms_per_step": times[False] * 1e3,
            "filtered_over_unfiltered": times[True] / times[False],
            "update_ms": upd[True], "unfiltered_update_ms": upd[False],
            "update_filtered_over_unfiltered": upd[True] / upd[False], "estimate": res["value"]}


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


def bench_subq(dev, stream, steps, calls=4, m=1 << 18, d=15):
    """Sub-query sketches for a join-order search (Sec. 3.4): every connected sub-chain
    of the 5-chain (10 sub-queries), 4 calls of 2^20 tuples per relation, Zipf(1.0) over
    10^7, m = 2^18, d = 15.  One pass per relation fills the 11 distinct sketches
    (cs_subq_update), then one batched estimate of all sub-queries; beside it the plain
    path builds one query handle per sub-query (30 relation sketches, each relation's
    keys read once per sub-query it is in, its kept columns prepared beforehand) and
    estimates them one by one."""
    import torch

    import paper_2402_15953_amd as csk
    import workloads as W
    g = W.chain(5)
    masks = W.connected_subqueries(g)
    n_call = 1 << 20
    n = calls * n_call
    keys = [W.relation_keys(g, k, n, "zipf", config=3, s=1.0, D=10 ** 7, device=dev).to(torch.int32).contiguous()
            for k in range(g.n_rel)]
    sq = csk.SubQueries(g, masks, m, d, 21)
    n_targets, _ = sq.layout()
    plain = []
    for mk in masks:
        gq, rels, cols = W.subquery_graph(g, mk)
        sub_keys = [keys[k][:, c].contiguous() for k, c in zip(rels, cols)]
        plain.append((csk.Sketch(gq, m, d, 21), sub_keys))
    torch.cuda.synchronize()

    def subq_step(ev=None):
        sq.reset(stream=stream)
        for k in range(g.n_rel):
            for c in range(calls):
                sq.update(k, keys[k][c * n_call:(c + 1) * n_call], stream=stream)
        if ev:
            ev.record(stream)
        return sq.estimate_all(stream=stream)

    def plain_step(ev=None):
        for sk, sub_keys in plain:
            sk.reset(stream=stream)
            for i, kk in enumerate(sub_keys):
                for c in range(calls):
                    sk.update(i, kk[c * n_call:(c + 1) * n_call], None, stream=stream)
        if ev:
            ev.record(stream)
        return [sk.estimate(stream=stream) for sk, _ in plain]

    res = {}
    with torch.cuda.stream(stream):
        for name, fn in (("subq", subq_step), ("plain", plain_step)):
            fn()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(steps):
                fn()
            torch.cuda.synchronize()
            dt = (time.perf_counter() - t0) / steps
            ta, tb = csk.Timer(), csk.Timer()
            ta.record(stream)
            fn(tb)
            torch.cuda.synchronize()
            res[name] = (dt, ta.elapsed_ms(tb))
    sq.close()
    for sk, _ in plain:
        sk.close()
    total = n * g.n_rel
    return {"workload": "all 10 connected sub-chains of the 5-chain, 4 x 2^20 tuples per relation, "
                        f"Zipf(1.0) over 1e7, m={m}, d={d}",
            "sub_queries": len(masks), "targets": n_targets,
            "plain_relation_sketches": sum(len(W.subquery_graph(g, mk)[1]) for mk in masks),
            "base_tuples_per_step": total,
            "subq_tuples_per_s": total / res["subq"][0], "plain_tuples_per_s": total / res["plain"][0],
            "speedup": res["plain"][0] / res["subq"][0],
            "subq_ms_per_step": res["subq"][0] * 1e3, "plain_ms_per_step": res["plain"][0] * 1e3,
            "subq_update_ms": res["subq"][1], "plain_update_ms": res["plain"][1]}


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
    identical = est_batch == est_plain
    # the autotuner: task kind and chunk per item class, split per transform length;
    # then the same batch planned and estimated with the tuned table
    csk.tune_clear()
    t0 = time.perf_counter()
    trep = b.tune(items, stream=stream)
    splits = {}
    for L in sorted({(sp.m - 1).bit_length() for sp in specs}):
        if L > 12:
            splits[L] = csk.tune_transform(L, n_vec=64, stream=stream)["best"]["split"]
    t_tune = time.perf_counter() - t0
    reset_all()
    b.capture(items, stream=stream)
    b.replay(stream=stream)
    torch.cuda.synchronize()
    b.estimate(sks, stream=stream)
    reset_all()
    t0 = time.perf_counter()
    b.replay(stream=stream)
    torch.cuda.synchronize()
    t_up_tuned = time.perf_counter() - t0
    t0 = time.perf_counter()
    est_tuned = b.estimate(sks, stream=stream)
    t_est_tuned = time.perf_counter() - t0
    stats_tuned = b.stats()
    csk.tune_clear()
    b.close()
    for sk_ in sks:
        sk_.close()
    return {"workload": f"{n_queries} chain/star queries, 2-6 relations, n log-uniform [1e3,1e6], "
                        "m=2^10..2^16, d in {5,9}, Zipf(1.2) over 1e6, weights +1",
            "tuples": tuples,
            "plain_update_tuples_per_s": tuples / t_up_plain, "batched_update_tuples_per_s": tuples / t_up_batch,
            "plain_estimates_per_s": n_queries / t_est_plain, "batched_estimates_per_s": n_queries / t_est_batch,
            "update_speedup": t_up_plain / t_up_batch, "estimate_speedup": t_est_plain / t_est_batch,
            "batched_plan_s": t_plan, "tasks": stats, "identical_estimates": identical,
            "tuned": {"update_tuples_per_s": tuples / t_up_tuned, "estimates_per_s": n_queries / t_est_tuned,
                      "update_over_rule": t_up_batch / t_up_tuned, "estimate_over_rule": t_est_batch / t_est_tuned,
                      "classes": trep["classes"], "rejected": trep["rejected"],
                      "class_sum_rule_ms": trep["rule_ms"], "class_sum_tuned_ms": trep["tuned_ms"],
                      "splits": splits, "tuning_s": t_tune, "tasks": stats_tuned,
                      "identical_estimates": est_tuned == est_plain}}


def bench_serving(n_queries, dev, seconds, rates, stream):
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
    plain_sks = [csk.Sketch(sp.graph, sp.m, sp.d, sp.sketch_seed) for sp in specs]
    with torch.cuda.stream(stream):
        for qi, sp in enumerate(specs):  # the same warm-up as the served queries
            plain_sks[qi].update(0, pools[qi][0][:1024], ones[:1024], stream=stream, unit_weights=True)
            plain_sks[qi].estimate(stream=stream)
            plain_sks[qi].update(0, pools[qi][0][:1024], minus[:1024], stream=stream, unit_weights=True)
    torch.cuda.synchronize()
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
        est_ticket = {}
        for ri, (ta, kind, q, k, off, ln, sign) in enumerate(plan):
            while time.perf_counter() - t0 < ta:
                pass
            try:
                if kind == "U":
                    srv.submit_update(qids[q], k, pools[q][k][off:off + ln],
                                      (ones if sign > 0 else minus)[off:off + ln], unit_weights=True)
                    tuples += ln
                else:
                    est_ticket[srv.submit_estimate(qids[q])] = ri
            except csk.CsError:
                busy += 1
        srv.drain()
        wall = time.perf_counter() - t0
        comps = srv.poll(1 << 20)
        lat_u = np.array([c["done_us"] - c["submit_us"] for c in comps if c["kind"] == 0]) / 1e3
        lat_e = np.array([c["done_us"] - c["submit_us"] for c in comps if c["kind"] == 1]) / 1e3
        n_e = int(len(lat_e))
        served_est = {est_ticket[c["ticket"]]: c["estimate"]["value"] for c in comps
                      if c["kind"] == 1 and c["ticket"] in est_ticket}

        def pct(a, p):
            return float(np.percentile(a, p)) if len(a) else None

        progress("serving window at %g batches/s done%s" % (rate, " (warm-up)" if li == 0 else ""))
        # the plain per-query path on the same trace: one handle per query (same seeds,
        # so the same hash functions), each request issued at its arrival time in order,
        # updates asynchronous on one stream, estimates synchronous (cs_estimate)
        plain_lv = replay_plain(plan, plain_sks, pools, ones, minus, stream)
        same = all(plain_lv["estimates"].get(ri) == v for ri, v in served_est.items())
        progress("plain window at %g batches/s done" % rate)
        if li == 0:
            continue
        levels.append({"offered_update_batches_per_s": rate, "offered_estimates_per_s": rate / 4,
                       "seconds": wall, "tuples_per_s": tuples / wall, "estimates_per_s": n_e / wall,
                       "update_p50_ms": pct(lat_u, 50), "update_p99_ms": pct(lat_u, 99),
                       "estimate_p50_ms": pct(lat_e, 50), "estimate_p99_ms": pct(lat_e, 99),
                       "requests": len(comps), "refused": busy,
                       "plain": {k: v for k, v in plain_lv.items() if k != "estimates"},
                       "identical_estimates": bool(same and len(served_est) == n_e)})
    st = srv.stats()
    srv.close()
    for sk_ in plain_sks:
        sk_.close()
    return {"workload": f"{n_queries} live chain/star queries, m=2^14..2^18, d=9, Zipf(1.1) over 1e6, "
                        "update batches 2^U[10,18] tuples, 10% deletes, estimate:update = 1:4, Poisson arrivals",
            "resident_counter_bytes": int(st["used_bytes"]), "levels": levels,
            "update_launches": int(st["update_launches"]), "estimate_batches": int(st["estimate_batches"])}


def replay_plain(plan, sks, pools, ones, minus, stream):
    """One serving window on the plain per-query path: requests in arrival order, each
    issued no earlier than its arrival; an update's completion is a timing event recorded
    behind it on the stream, an estimate's the return of the synchronous cs_estimate."""
    import numpy as np
    import torch
    # the reference event completes before the window's clock starts, so the device
    # times of later events measured from it are never earlier than the host's
    ev0 = torch.cuda.Event(enable_timing=True)
    ev0.record(stream)
    ev0.synchronize()
    t0 = time.perf_counter()
    lat_u, lat_e, ev_u, ests = [], [], [], {}
    tuples = 0
    with torch.cuda.stream(stream):
        for ri, (ta, kind, q, k, off, ln, sign) in enumerate(plan):
            while time.perf_counter() - t0 < ta:
                pass
            if kind == "U":
                sks[q].update(k, pools[q][k][off:off + ln], (ones if sign > 0 else minus)[off:off + ln],
                              stream=stream, unit_weights=True)
                ev = torch.cuda.Event(enable_timing=True)
                ev.record(stream)
                ev_u.append((ta, ev))
                tuples += ln
            else:
                e = sks[q].estimate(stream=stream)
                lat_e.append((time.perf_counter() - t0 - ta) * 1e3)
                ests[ri] = e["value"]
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    for ta, ev in ev_u:
        lat_u.append(ev0.elapsed_time(ev) - ta * 1e3)

    def pct(a, p):
        return float(np.percentile(np.array(a), p)) if len(a) else None

    return {"seconds": wall, "tuples_per_s": tuples / wall, "estimates_per_s": len(lat_e) / wall,
            "update_p50_ms": pct(lat_u, 50), "update_p99_ms": pct(lat_u, 99),
            "estimate_p50_ms": pct(lat_e, 50), "estimate_p99_ms": pct(lat_e, 99), "estimates": ests}


def cpu_baseline(host_keys):
    """The oracle (plain C Alg. 2 loop) on a prefix of the headline input (Zipf 1.0),
    on this host: one thread on one 2^20-tuple slice per relation, and one thread per
    core of this process's CPU share (at most 16) on more slices, each thread sketching
    its own slices into private counters that are then summed (the sketch is linear,
    Sec. 2.2).  The exact estimate of one repetition (number-theoretic transforms of
    2^18 points) is timed once and reported per estimate of all d repetitions."""
    import platform
    from concurrent.futures import ThreadPoolExecutor

    import numpy as np

    import oracle
    import workloads as W

    graph = W.chain(5)
    m, d, seed = 1 << 18, 15, 8
    n_call = 1 << 20
    info = oracle.analyze(graph)
    co = oracle.draw_coefficients(seed, d, len(info.edges), info.n_comp)
    host = [k.numpy().view(np.uint32).reshape(k.shape[0], -1) for k in host_keys]
    slices = host[0].shape[0] // n_call
    t0 = time.perf_counter()
    one = [oracle.create_sketch(info, k, host[k][:n_call], None, m, co) for k in range(graph.n_rel)]
    t1 = time.perf_counter()
    try:
        share = len(os.sched_getaffinity(0))
    except AttributeError:
        share = os.cpu_count() or 1
    threads = max(1, min(16, share))
    jobs = [(k, i) for k in range(graph.n_rel) for i in range(slices)]
    t2 = time.perf_counter()
    with ThreadPoolExecutor(max_workers=threads) as ex:
        parts = list(ex.map(lambda ki: (ki[0], oracle.create_sketch(info, ki[0], host[ki[0]][ki[1] * n_call:(ki[1] + 1) * n_call],
                                                                    None, m, co)), jobs))
    sums = [np.zeros((d, m), dtype=np.int64) for _ in range(graph.n_rel)]
    for k, sk in parts:
        sums[k] += sk
    t3 = time.perf_counter()
    t4 = time.perf_counter()
    oracle.estimate_alg3(info, [one[k][0] for k in range(graph.n_rel)], m, method="ntt")
    t5 = time.perf_counter()
    model = ""
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        model = platform.processor()
    tuples1 = n_call * graph.n_rel
    tuplesn = n_call * slices * graph.n_rel
    return {"value": tuples1 / (t1 - t0), "unit": "tuple updates/s", "cores": 1, "kind": "oracle",
            "sample": f"first 2^20 tuples of each of the 5 relations of the Zipf(1.0) stream (m=2^18, d=15), "
                      f"one thread: {t1 - t0:.2f} s",
            "threaded": {"value": tuplesn / (t3 - t2), "cores": threads,
                         "sample": f"first {slices} x 2^20 tuples of each relation, {len(jobs)} slices over "
                                   f"{threads} threads with private sketches summed: {t3 - t2:.2f} s"},
            "estimate_s_per_repetition": t5 - t4, "estimates_per_s": 1.0 / ((t5 - t4) * d),
            "nproc": os.cpu_count(), "cpu_share": share, "cpu_model": model}


if __name__ == "__main__":
    main()
