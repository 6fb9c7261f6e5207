"""Benchmark of the sketch update + estimate hot path on one MI355X.

Workload (the metric's configuration): a 3-relation chain R1(A) - R2(A, B) - R3(B),
10^7 tuples per relation, uint32 keys Zipf(s = 1.1) over a domain of 10^6 per
attribute, m = 2^16 buckets, d = 9 repetitions, int64 counters, weights +1.  Keys are
generated on the GPU and resident in HBM before timing.

One step = the whole plain hot path over one batch: zero the counters, stream every
relation's tuples into its d x m sketches (one update launch per relation), then the
estimate (fp64 FFT spectral product-reduce, exactness step, median over d).

Printed: one JSON line.  `value` is tuple updates per second over whole steps.
`roofline` describes the dominant kernel (the update of the two-column relation),
timed with HIP events on the stream it runs on.  `cpu_baseline` is the CPU oracle on a
bounded prefix of the same input, on this host.
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
# issues 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz = 3.93e13 VALU lane-instructions/s,
# and the compiled step is 13 VALU instructions (2 v_mad_u64_u32, 64-bit adds and
# shifts, the Mersenne fold), so 3.02e12 steps/s.
ALU_STEP_PEAK = 256 * 4 * 16 * 2.4e9 / 13.0


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--n", type=int, default=10 ** 7, help="tuples per relation")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--cpu-tuples", type=int, default=1 << 22, help="oracle sample per relation")
    ap.add_argument("--strategy", type=int, default=0)
    return ap.parse_args()


def horner_steps_per_tuple(graph, k, d):
    """d * sum over key columns (1 bin step + 3 steps per join at that attribute)."""
    steps = 0
    for u in graph.columns(k):
        joins = sum(1 for e in graph.edges if u in e)
        steps += 1 + 3 * joins
    return d * steps


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU; --gpus %d is not supported" % args.gpus}))
        print("bench.py runs on exactly one GPU (no multi-GPU path in this build)", file=sys.stderr)
        sys.exit(2)

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
    est_ev = []

    def step(record):
        sk.reset(stream=stream)
        for k in range(n_rel):
            if record:
                a = torch.cuda.Event(enable_timing=True)
                b = torch.cuda.Event(enable_timing=True)
                a.record(stream)
            sk.update(k, keys[k], None, stream=stream, strategy=args.strategy)
            if record:
                b.record(stream)
                ev[k].append((a, b))
        if record:
            a = torch.cuda.Event(enable_timing=True)
            b = torch.cuda.Event(enable_timing=True)
            a.record(stream)
        res = sk.estimate(stream=stream)
        if record:
            b.record(stream)
            est_ev.append((a, b))
        return res

    with torch.cuda.stream(stream):
        for _ in range(args.warmup):
            step(False)
        torch.cuda.synchronize()
        t_start = time.perf_counter()
        for _ in range(args.steps):
            res = step(True)
        torch.cuda.synchronize()
        elapsed = time.perf_counter() - t_start

    ms_per_step = elapsed * 1e3 / args.steps
    tuples_per_step = n * n_rel
    value = tuples_per_step * args.steps / elapsed
    upd_ms = {k: sum(a.elapsed_time(b) for a, b in ev[k]) / len(ev[k]) for k in range(n_rel)}
    est_ms = sum(a.elapsed_time(b) for a, b in est_ev) / len(est_ev)
    upd_total_ms = sum(upd_ms.values())

    # dominant kernel: the slowest relation's update launch
    kdom = max(upd_ms, key=upd_ms.get)
    a_dom = len(graph.columns(kdom))
    bytes_dom = n * 4 * a_dom                       # uint32 keys, weights NULL
    steps_dom = n * horner_steps_per_tuple(graph, kdom, d)
    dur_s = upd_ms[kdom] / 1e3
    alu_achieved = steps_dom / dur_s
    hbm_achieved = bytes_dom / dur_s / 1e9

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
                     "unit": "T Horner-steps/s", "frac": alu_achieved / ALU_STEP_PEAK, "traffic": None,
                     "kernel": f"update relation {kdom} ({a_dom} key columns)",
                     "hbm_GBps": hbm_achieved, "hbm_frac": hbm_achieved / HBM_PEAK_GBS},
        "update_ms_per_relation": {str(k): v for k, v in upd_ms.items()},
        "update_tuples_per_s": tuples_per_step / (upd_total_ms / 1e3),
        "estimate_ms": est_ms,
        "estimates_per_s": 1e3 / est_ms,
        "init_ms": init_ms,
        "estimate": {"value": res["value"], "exact": res["exact"], "n_modular": res["n_modular"]},
    }

    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(graph, keys, m, d, seed, args.cpu_tuples)

    print(json.dumps(out), flush=True)
    sk.close()


def cpu_baseline(graph, keys, m, d, seed, n_sample):
    """The oracle (plain C sketch loop + exact NTT estimate) on the first n_sample
    tuples of every relation: tuples per second of the same step on this host."""
    import numpy as np

    import oracle

    info = oracle.analyze(graph)
    co = oracle.draw_coefficients(seed, d, len(info.edges), info.n_comp)
    host = [k[:n_sample].cpu().numpy().view(np.uint32) for k in keys]
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
