#!/usr/bin/env python3
"""Benchmark of the exact sign-vector sum on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload NAME]

A step is one complete exact count of every instance in the workload (plan,
kernel launches, host CRT).  Prints one JSON line on stdout; progress goes to
stderr.

Workloads (all inputs are the problem statements themselves: no data files):
  batch  Skolem n = 16, 17, 20, 21; Langford n = 15, 16, 19, 20; hooked n = 14, 15
         (the default: the mixed-instance run the metric's n = 20 figures come from)
  s24    Skolem n = 24, 2^47 sign vectors (the paper's single-GPU headline count)
  l24    Langford n = 24
  s20    Skolem n = 20;  l20  Langford n = 20
  s12    Skolem n = 12, two primes (the small correctness case)
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "sign-vector terms/s for exact S(n),L(n) at n=20,24; PT rel. error vs GPU-s"
PEAK_LANE_OPS = 256 * 64 * 2.4e9  # MI355X: 256 CUs x 64 lanes x 2.4 GHz full-rate VALU lane-ops/s

WORKLOADS = {
    "batch": [("skolem", 16), ("skolem", 17), ("skolem", 20), ("skolem", 21), ("langford", 15),
              ("langford", 16), ("langford", 19), ("langford", 20), ("hooked", 14), ("hooked", 15)],
    "s24": [("skolem", 24)],
    "l24": [("langford", 24)],
    "s20": [("skolem", 20)],
    "l20": [("langford", 20)],
    "s12": [("skolem", 12)],
}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def expected_values():
    """Printed values (Tables 7, 8) and stored oracle counts, for the check."""
    out = {}
    with open(os.path.join(ROOT, "tests", "golden", "paper_counts.json")) as f:
        paper = json.load(f)
    for v in ("skolem", "langford"):
        for n, val in paper[v].items():
            if not n.startswith("_"):
                out[(v, int(n))] = int(val)
    path = os.path.join(ROOT, "tests", "golden", "oracle_counts.json")
    if os.path.exists(path):
        with open(path) as f:
            g = json.load(f)
        for key, rec in g.items():
            if key.startswith("_"):
                continue
            v, n = key.split(":")
            if v == "hooked":
                out[(v, int(n))] = int(rec["ordered"])
    return out


def alg_ops_per_term(desc) -> int:
    """Minimal VALU lane-operations per sign vector for this representation:
    n pair-sum updates, n - 1 exact multiplications, and per prime one
    accumulate pair (2) plus 4 per double-word modular reduction (quotient
    estimate 2, fma, low-part add) for each of the G - 1 group products."""
    n = sum(1 for s in desc["slot_factor"] if s >= 0)
    P, G = desc["primes_used"], desc["groups"]
    return n + (n - 1) + P * (4 * max(G - 1, 0) + 2 + (3 if G == 1 else 0))


def cpu_baseline(instances, threads):
    """The CPU oracle's Gray-code partial sum, timed on a bounded slice of the
    workload's largest instance (about 10-30 s of host work)."""
    import oracle as O
    O.build(force=False)
    variant, n = max(instances, key=lambda vn: vn[1])
    pos, _ = O.instance(n, variant)
    free_bits = 28 if n >= 20 else 26
    fixed = {pos[0]: 1}
    for q in pos[1 + free_bits:]:
        fixed[q] = 1
    terms = 1 << (len(pos) - len(fixed))
    p = O.primes_below(1 << 46, 1)[0]
    t0 = time.time()
    O.chunk_partial(n, variant, fixed, p, "gray", threads=threads)
    dt = time.time() - t0
    return {"value": terms / dt, "unit": "terms/s", "cores": threads, "kind": "oracle",
            "sample": f"{variant} n={n}: Gray-code partial sum over 2^{len(pos) - len(fixed)} sign vectors "
                      f"(x at positions above {pos[free_bits]} fixed), one prime, {threads} threads, "
                      f"{dt:.1f} s"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="batch", choices=sorted(WORKLOADS))
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--log2-chunk", type=int, default=0)
    ap.add_argument("--kernel", type=int, default=0)
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: this build runs on one GPU only (asked for --gpus {args.gpus}); "
              "the exact sum shards by chunk ranges across GPUs, see DESIGN.md", file=sys.stderr)
        sys.exit(2)

    import paper_1507_00315_amd as sk
    try:
        import torch
        sync = torch.cuda.synchronize if torch.cuda.is_available() else (lambda: None)
    except Exception:  # torch is plumbing only
        sync = lambda: None  # noqa: E731

    instances = WORKLOADS[args.workload]
    tuning = {"log2_chunk_terms": args.log2_chunk, "kernel": args.kernel}
    if args.workload == "s12":
        tuning["primes"] = 2
    want = expected_values()

    def step(tag):
        res = []
        for v, n in instances:
            r = sk.count_ex(n, v, ordered=(v == "hooked"), tuning=tuning)
            ok = want.get((v, n))
            res.append((v, n, r.count, r.stats, None if ok is None else (ok == r.count)))
            log(f"[{tag}] {v} n={n}: {r.count}  kernel {r.stats['kernel_ms']:.1f} ms  "
                f"{r.stats['terms'] / max(r.stats['kernel_ms'], 1e-9) * 1e3:.3e} terms/s  "
                f"check={res[-1][4]}")
        return res

    for w in range(args.warmup):
        step(f"warmup {w}")
    sync()
    t0 = time.perf_counter()
    results = []
    for s in range(args.steps):
        results.append(step(f"step {s}"))
    sync()
    elapsed = time.perf_counter() - t0

    terms_per_step = sum(r[3]["terms"] for r in results[0])
    total_terms = terms_per_step * args.steps
    value = total_terms / elapsed
    all_ok = all(r[4] is not False for st in results for r in st)

    # Roofline of the exact kernel: algorithmic lane-ops per launch over the
    # launch durations measured with HIP events on the launch stream.
    alg = 0.0
    kms = 0.0
    launches = 0
    for st in results:
        for v, n, _c, stats, _ok in st:
            d = sk.describe(n, v)
            d["primes_used"] = stats["nprimes"]
            alg += stats["terms"] * alg_ops_per_term(d)
            kms += stats["kernel_ms"]
            launches += stats["launches"]
    achieved = alg / (kms * 1e-3) if kms > 0 else 0.0
    kernel_name = sk.kernel_name(results[0][0][3]["kernel_variant"])

    line = {
        "metric": METRIC,
        "value": value,
        "unit": "terms/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": elapsed * 1e3 / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": args.workload,
                   "instances": [f"{v}:{n}" for v, n in instances],
                   "terms_per_step": terms_per_step,
                   "primes_per_instance": {f"{r[0]}:{r[1]}": r[3]["nprimes"] for r in results[0]},
                   "log2_chunk_terms": {f"{r[0]}:{r[1]}": r[3]["log2_chunk_terms"] for r in results[0]},
                   "results_match_expected": all_ok},
        "roofline": {"bound": "alu", "achieved": achieved, "peak": PEAK_LANE_OPS, "unit": "lane-op/s",
                     "frac": achieved / PEAK_LANE_OPS, "traffic": None, "kernel": kernel_name,
                     "launches": launches, "avg_launch_ms": kms / max(launches, 1)},
    }
    if not args.no_cpu_baseline:
        threads = min(16, os.cpu_count() or 1)
        log("cpu baseline ...")
        line["cpu_baseline"] = cpu_baseline(instances, threads)
    print(json.dumps(line), flush=True)
    if not all_ok:
        sys.exit(1)


if __name__ == "__main__":
    main()
