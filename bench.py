#!/usr/bin/env python3
"""Benchmark of the exact sign-vector sum on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload NAME]

A step is one complete exact count of every instance in the workload (plan,
kernel launches, host CRT).  Prints one JSON line on stdout; progress goes to
stderr.

Workloads (all inputs are the problem statements themselves: no data files):
  mixed  (the default) one step = the batch below in one persistent launch, then
         the n = 24 slices: 8192 seeded chunks of 2^26 sign vectors of Skolem
         n = 24 and of Langford n = 24 (two primes, the ones a full count uses),
         16 rows of each checked against the oracle's stored recomputation
  batch  Skolem n = 16, 17, 20, 21; Langford n = 15, 16, 19, 20; hooked n = 14, 15
         (the mixed-instance run the metric's n = 20 figures come from)
  s24    Skolem n = 24, 2^47 sign vectors (the paper's single-GPU headline count)
  l24    Langford n = 24
  s20    Skolem n = 20;  l20  Langford n = 20
  s12    Skolem n = 12, two primes (the small correctness case)
  s25    Skolem n = 25 (2^49 sign vectors; the paper used four GPUs)
  all24  every nonzero S(n) and L(n) with n <= 24 in one batched call (one
         persistent launch per batched group; n <= 11 by separate launches)
  pt     the tempering curve alone (the plain runs' level-moves/s as the value)
  larsen20  S(20) and L(20) by inclusion-exclusion over the empty positions
         (the third approach of Sec. 2; 2^40 terms each, no symmetry)
  l28slice  Langford n = 28: a seeded 1/4096 subset of its 2^24 prefix chunks
         (2^43 sign vectors) with the three primes a full count needs; the
         projected full-count time is reported
"""
from __future__ import annotations

import argparse
import json
import os
import subprocess
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "sign-vector terms/s for exact S(n),L(n) at n=20,24; PT rel. error vs GPU-s"
PEAK_LANE_OPS = 256 * 64 * 2.4e9  # MI355X: 256 CUs x 4 SIMD x 16 lanes x 2.4 GHz: VALU lane-instructions/s

WORKLOADS = {
    "mixed": [("skolem", 16), ("skolem", 17), ("skolem", 20), ("skolem", 21), ("langford", 15),
              ("langford", 16), ("langford", 19), ("langford", 20), ("hooked", 14), ("hooked", 15)],
    "batch": [("skolem", 16), ("skolem", 17), ("skolem", 20), ("skolem", 21), ("langford", 15),
              ("langford", 16), ("langford", 19), ("langford", 20), ("hooked", 14), ("hooked", 15)],
    "s24": [("skolem", 24)],
    "l24": [("langford", 24)],
    "s20": [("skolem", 20)],
    "l20": [("langford", 20)],
    "s12": [("skolem", 12)],
    "l28slice": [("langford", 28)],
    "pt": [],
    "s25": [("skolem", 25)],
    # the inclusion-exclusion count (third approach of Sec. 2) of S(20) and L(20)
    "larsen20": [("skolem", 20), ("langford", 20)],
    # every nonzero S(n) and L(n) up to n = 24 (existence: S needs n = 0, 1 mod 4,
    # L needs n = 0, 3 mod 4), largest first
    "all24": sorted([("skolem", n) for n in range(1, 25) if n % 4 in (0, 1)] +
                    [("langford", n) for n in range(1, 25) if n % 4 in (0, 3)], key=lambda x: -x[1]),
}
L28_CHUNK_BITS, L28_SLICE = 24, 4096


# HBM bytes per launch from rocprofv3 --pmc FETCH_SIZE / WRITE_SIZE runs (KiB per
# dispatch), scaled by what the same counters read for a plain 1 GiB device copy
# (FETCH_SIZE x 2.0, WRITE_SIZE x 1.0).  Valid only for the kernel sources they
# were taken on: the fingerprint is a SHA-256 over those sources with comments
# removed, and a changed kernel reports traffic null until the counters are
# taken again.
KERNEL_SOURCES = {
    "exact_batch_kernel": ["exact_batch.hip", "sk_batch.h", "exact_v2_body.h", "exact_common.h", "sk_plan.h",
                           "sk_internal.h"],
    "exact_v2_kernel": ["exact_v2_inst.hip", "exact_v2_body.h", "exact_common.h", "sk_plan.h", "sk_internal.h"],
}
MEASURED_TRAFFIC = {
    # (kernel, workload or leg, log2 sign vectors per work item, waves per launch):
    #     (fingerprint, FETCH_SIZE KiB, WRITE_SIZE KiB)
    ("exact_batch_kernel", "batch", 22, 6144): ("30f4c6bb20835127", 1247.125, 13246.46875),
    ("exact_batch_kernel", "batch", 22, 8192): ("30f4c6bb20835127", 1249.1875, 13311.375),
    ("exact_v2_kernel", "skolem:24 slice", 26, 8192): ("fcb120309dc22ca1", 628.9375, 24832.0),
    ("exact_v2_kernel", "langford:24 slice", 26, 8192): ("fcb120309dc22ca1", 613.1875, 24832.0),
}
FETCH_FACTOR, WRITE_FACTOR = 2.0, 1.0


def kernel_fingerprint(kernel: str) -> str:
    """SHA-256 over the kernel's sources with comments removed and white space
    collapsed (a change of a comment or of layout does not change the kernel;
    any change of code does)."""
    import hashlib
    import re
    h = hashlib.sha256()
    for name in KERNEL_SOURCES.get(kernel, []):
        with open(os.path.join(ROOT, "paper_1507_00315_amd", "csrc", name), encoding="utf-8") as f:
            text = f.read()
        text = re.sub(r"/\*.*?\*/", " ", text, flags=re.S)
        text = re.sub(r"//[^\n]*", " ", text)
        h.update(" ".join(text.split()).encode())
    return h.hexdigest()[:16]


def traffic_per_launch(kernel: str, workload: str, log2_chunk: int, waves: int):
    rec = MEASURED_TRAFFIC.get((kernel, workload, log2_chunk, waves))
    if rec is None or rec[0] != kernel_fingerprint(kernel):
        return None
    return (rec[1] * FETCH_FACTOR + rec[2] * WRITE_FACTOR) * 1024


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


def valu_per_term(desc) -> int:
    """VALU instructions the tuned kernel issues per sign vector (design count):
    NP packed adds A + B, NQ packed pair products, NQ SDWA quad products, NQ
    conversions to fp64, NQ - G exact group products, the exact high/low split
    of g0 g1 (G >= 2), and per prime 4 residue/accumulate instructions (plus
    one low-part add shared by all primes for G >= 2).  With G >= 3 groups the
    kernel runs the two-group chain on g0 and the product of the other groups
    (one more group product, two range checks) and evaluates a job again with
    the full chain only when a term left that chain's exact range, which the
    largest products alone do: the count is the two-group one."""
    nq, G, P = desc["quads"], desc["groups"], desc["primes_used"]
    np_ = 2 * nq
    if G == 1:
        return np_ + 3 * nq + (nq - 1) + 4 * P
    if G == 2:
        return np_ + 3 * nq + (nq - 2) + 2 + 4 * P + 1
    return np_ + 3 * nq + (nq - 2) + 2 + 2 + 4 * P + 1


def ring_ops_per_term(n: int, P: int) -> int:
    """The method's own work per sign vector: n pair-sum updates, n - 1
    modular multiplications and one accumulate per prime."""
    return n + P * (n - 1) + P


def n24_slices():
    """The n = 24 slices of the default step: for Skolem and Langford n = 24,
    8192 seeded chunks of 2^26 sign vectors (of 2^21), with the two primes a
    full count uses, and the rows the oracle recomputed for 16 of them
    (tests/golden/big_chunks.json, written by tests/golden/make_big_chunks.py)."""
    from paper_1507_00315_amd import inputs
    with open(os.path.join(ROOT, "tests", "golden", "big_chunks.json")) as f:
        g = json.load(f)
    out = []
    for v in ("skolem", "langford"):
        c = g["cases"][f"{v}:24"]
        seed = inputs.N24_SLICE_SEEDS[v]
        ids = inputs.distinct_ids(seed, inputs.N24_CHUNK_BITS, inputs.N24_SLICE)
        pos = {cid: i for i, cid in enumerate(ids)}
        check = [(pos[ch["id"]], [int(x) for x in ch["residues"]]) for ch in c["chunks"]]
        out.append({"variant": v, "seed": seed, "log2_chunks": inputs.N24_CHUNK_BITS, "ids": ids,
                    "primes": [int(p) for p in g["primes"]], "check": check})
    return out


def host_threads():
    """Threads the CPU baseline uses: the host cores this process may run on
    (its affinity mask), capped by OMP_NUM_THREADS where the machine sets it
    (a GPU machine gives one GPU's jobs a share of its cores that way)."""
    try:
        aff = len(os.sched_getaffinity(0))
    except (AttributeError, OSError):
        aff = os.cpu_count() or 1
    omp = os.environ.get("OMP_NUM_THREADS", "")
    return min(aff, int(omp)) if omp.isdigit() and int(omp) > 0 else aff


def host_info():
    info = {"cpu": cpu_model(), "os_cpu_count": os.cpu_count(),
            "OMP_NUM_THREADS": os.environ.get("OMP_NUM_THREADS")}
    try:
        info["affinity_cpus"] = len(os.sched_getaffinity(0))
    except (AttributeError, OSError):
        pass
    try:
        import subprocess
        info["nproc"] = int(subprocess.run(["nproc"], capture_output=True, text=True, timeout=10).stdout.strip())
        info["nproc_all"] = int(subprocess.run(["nproc", "--all"], capture_output=True, text=True,
                                               timeout=10).stdout.strip())
    except Exception:  # nproc missing: the counts above remain
        pass
    return info


def cpu_baseline(instances):
    """The CPU oracle as it stands, on the GPU machine's host cores: its Gray-code
    partial sum on a bounded slice of the workload's largest instance (about
    10-30 s of host work), and its backtracking count (the plain definition,
    largest difference first) of S(12) and S(13)."""
    import oracle as O
    O.build(force=False)
    threads = host_threads()
    variant, n = max(instances, key=lambda vn: vn[1])
    pos, _ = O.instance(n, variant)
    free_bits = 32 if n >= 20 else 28
    fixed = {pos[0]: 1}
    for q in pos[1 + free_bits:]:
        fixed[q] = 1
    terms = 1 << (len(pos) - len(fixed))
    p = O.primes_below(1 << 46, 1)[0]
    t0 = time.time()
    O.chunk_partial(n, variant, fixed, p, "gray", threads=threads)
    dt = time.time() - t0
    bt = []
    for bn in (12, 13):
        t1 = time.time()
        c = O.count_backtrack(bn, "skolem", threads=threads)
        d1 = time.time() - t1
        bt.append({"instance": f"skolem:{bn}", "ordered_count": c, "seconds": d1, "solutions_per_s": c / d1,
                   "threads": threads})
    return {"value": terms / dt, "unit": "terms/s", "cores": threads, "kind": "oracle", "host": host_info(),
            "sample": f"{variant} n={n}: Gray-code partial sum over 2^{len(pos) - len(fixed)} sign vectors "
                      f"(x at positions above {pos[free_bits]} fixed), one prime, {threads} threads, "
                      f"{dt:.1f} s",
            "backtracking": bt}


def geometric_ladder_49():
    """The 48 geometric replicas 0.05 * 120^(j/47), j = 0..47 (0.05 .. 6),
    below them the beta = 0 level whose samples give Z(beta_1) / Z(0); the
    terminal factor is the fraction of E = 0 samples at beta = 6."""
    return [0.0] + [0.05 * 120.0 ** (j / 47) for j in range(48)]


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


# The paper's own tempering estimates at its frontier (Table 7: S(28), S(29),
# exact values known, and S(32), S(33); Table 8: L(27), L(28), exact values
# known, and L(31), L(32)), for context beside ours.
PAPER_PT_ESTIMATES = {("skolem", 32): 2.213e26, ("skolem", 33): 3.614e27, ("langford", 31): 5.381e24,
                      ("langford", 32): 8.812e25, ("skolem", 28): 3.523e21, ("skolem", 29): 5.294e22,
                      ("langford", 27): 1.115e20, ("langford", 28): 1.603e21}


def pt_bench(sk, want, plain_iters, learned_iters, tuned_iters, ladders: int, learned_cfg: dict, seed: int = 1507,
             cpu_pt: bool = True):
    """Tempering estimates (Sec. 3): relative error against the printed S(20),
    S(24) and GPU seconds, as a curve over run lengths, for plain uniform moves
    on the 49-level ladder, with the learned proposal on the same ladder, and
    with plain moves on the ladder tuned by Sec. 3's rule (exchanges accepted
    at least half the time, as few levels as that takes); per curve the least
    GPU time that reached 1 % of exact; S(32), S(33), L(31), L(32) beside the
    paper's estimates.  Every run first burns in (learned: and trains on) a
    quarter of its recorded iterations; half_z is the equilibration check of
    each run (its two halves against each other)."""
    fixed = geometric_ladder_49()
    runs = []
    tuned = {}

    def one(variant, n, name, iters, betas):
        exact = want.get((variant, n))
        kw = dict(ladders=ladders, iterations=iters, seed=seed + n)
        if name == "learned":
            kw["proposal"] = sk.PROPOSAL_LEARNED
            kw["learned"] = dict(learned_cfg, train_iterations=iters // 4)
        else:
            kw["burn_in"] = iters // 4
        t0 = time.time()
        est, se, st = sk.approx(n, variant, betas, **kw)
        # gpu_s covers the burn-in (plain) or the sampling phase that feeds the
        # training (learned) too: a quarter of the recorded iterations more
        moves = st["moves"] + ladders * len(betas) * (iters // 4)
        rec = {"instance": f"{variant}:{n}", "n": n, "proposal": name, "levels": len(betas), "iterations": iters,
               "ladders": ladders, "estimate": est, "std_error": se, "rel_std_error": se / est if est else None,
               "half_z": st["half_z"], "gpu_s": st["gpu_ms"] * 1e-3, "wall_s": time.time() - t0,
               "level_moves": moves, "level_moves_per_gpu_s": moves / max(st["gpu_ms"] * 1e-3, 1e-12)}
        if exact:
            rec["exact"] = exact
            rec["rel_error"] = abs(est - exact) / exact
        paper = PAPER_PT_ESTIMATES.get((variant, n))
        if paper:
            rec["paper_estimate"] = paper
            rec["rel_diff_from_paper"] = (est - paper) / paper
        if name == "learned":
            j0 = learned_cfg["first_level"]
            rec.update({"train_gpu_s": st["train_ms"] * 1e-3, "learned_moves": st["learned_moves"],
                        "learned_accept_mean": sum(st["learned_accept"][j0:]) / (len(betas) - j0),
                        "plain_accept_mean_same_levels": sum(st["move_accept"][j0:]) / (len(betas) - j0),
                        "train_loss": st["train_loss"]})
        log(f"pt {name:7s} {variant}({n}) {len(betas)} levels 2^{iters.bit_length() - 1} it: {est:.6g} +- {se:.3g}"
            + (f"  rel err {rec['rel_error']:.2e}" if exact else "")
            + (f"  vs paper {rec['rel_diff_from_paper']:+.2%}" if paper else "")
            + f"  half_z {st['half_z']:+.1f}  gpu {rec['gpu_s']:.3f} s")
        runs.append(rec)

    sk.approx(20, "skolem", fixed, ladders=ladders, iterations=1 << 10, seed=seed)  # warm-up, not recorded
    for n in (20, 24):
        t0 = time.time()
        betas, acc = sk.pt_tune_ladder(n, "skolem", fixed[-1], target=0.5, max_levels=64, ladders=256,
                                       pilot_iterations=1 << 14, seed=seed)
        tuned[n] = {"betas": betas, "swap_accept": acc, "tuning_wall_s": time.time() - t0}
        log(f"tuned ladder S({n}): {len(betas)} levels, min exchange acceptance {min(acc):.3f} "
            f"({time.time() - t0:.1f} s)")
        # the same construction run on to 64 levels (the lowest acceptance split
        # first): a wavefront has 64 lanes, so levels up to 64 cost no time
        b64, acc64 = sk.pt_tune_ladder(n, "skolem", fixed[-1], target=0.999, max_levels=64, ladders=256,
                                       pilot_iterations=1 << 14, seed=seed)
        tuned[n]["betas_64"] = b64
        tuned[n]["swap_accept_64"] = acc64
        log(f"64-level ladder S({n}): min exchange acceptance {min(acc64):.3f}")
        for it in plain_iters:
            one("skolem", n, "plain", it, fixed)
        for it in learned_iters:
            one("skolem", n, "learned", it, fixed)
        for it in tuned_iters:
            one("skolem", n, "plain_tuned_ladder", it, betas)
        for it in tuned_iters:
            one("skolem", n, "plain_tuned_64", it, b64)
    # the frontier: the largest counts the paper has exactly (Table 4, Tables 7
    # and 8) and its estimates beyond them
    for variant, n in PAPER_PT_ESTIMATES:
        one(variant, n, "plain", plain_iters[-1], fixed)
    # per curve: the least GPU time whose estimate was within 1 % of exact
    to_1pct = {}
    for r in runs:
        if r.get("rel_error") is not None and r["rel_error"] <= 0.01:
            key = f"{r['instance']} {r['proposal']}"
            to_1pct[key] = min(to_1pct.get(key, float("inf")), r["gpu_s"])
    cpu = None
    if cpu_pt:
        import oracle as O
        O.build(force=False)
        iters = 1 << 20
        t0 = time.time()
        O.pt_ladder(32, "skolem", fixed, iters, seed, ladder=0, schedule="even_odd")
        dt = time.time() - t0
        cpu = {"value": iters * len(fixed) / dt, "unit": "level-moves/s", "cores": 1, "kind": "oracle",
               "cpu": cpu_model(), "sample": f"one ladder of S(32), {len(fixed)} levels, 2^20 iterations, {dt:.1f} s"}
    return {"ladder": "beta = 0, then 48 geometric levels 0.05 * 120^(j/47)", "levels": len(fixed),
            "tuned_ladders": tuned, "learned_config": {k: v for k, v in learned_cfg.items() if k != "params"},
            "runs": runs, "gpu_s_to_1pct": to_1pct, "cpu_baseline": cpu}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="mixed", choices=sorted(WORKLOADS))
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--log2-chunk", type=int, default=0)
    ap.add_argument("--kernel", type=int, default=0)
    ap.add_argument("--waves", type=int, default=0, help="waves per launch (with --log2-chunk)")
    ap.add_argument("--separate", action="store_true", help="batch workload as one launch per instance")
    ap.add_argument("--no-autotune", action="store_true")
    ap.add_argument("--no-pt", action="store_true", help="skip the tempering estimates")
    ap.add_argument("--pt-plain-log2", default="14,16,18,20,21", help="log2 recorded iterations, plain runs")
    ap.add_argument("--pt-learned-log2", default="16,18,20,21", help="log2 recorded iterations, learned runs")
    ap.add_argument("--pt-tuned-log2", default="18,20,21", help="log2 recorded iterations, tuned-ladder runs")
    ap.add_argument("--pt-ladders", type=int, default=1024)
    ap.add_argument("--pt-learned-every", type=int, default=256)
    ap.add_argument("--pt-learned-first", type=int, default=36)
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain device copy of 1 GiB (reference for the HBM byte counters)")
    ap.add_argument("--issue-calibration", action="store_true",
                    help="only run the vector-instruction issue-rate program (cost model of the tempering kernel)")
    args = ap.parse_args()
    if args.issue_calibration:
        probe = os.path.join(ROOT, "paper_1507_00315_amd", "issue_probe")
        if not os.path.exists(probe):
            sys.exit("bench.py: issue_probe is not built (python -m paper_1507_00315_amd.build)")
        sys.exit(subprocess.call([probe]))
    if args.copy_calibration:
        import torch
        src = torch.empty(1 << 28, dtype=torch.float32, device="cuda").fill_(1.0)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        log(f"copied {src.numel() * 4} bytes")
        return
    if args.gpus != 1:
        print(f"bench.py: this benchmark runs on one GPU only (asked for --gpus {args.gpus}); "
              "(the exact sum would shard by disjoint chunk-id ranges, one per GPU)", file=sys.stderr)
        sys.exit(2)

    import paper_1507_00315_amd as sk
    try:
        import torch
        sync = torch.cuda.synchronize if torch.cuda.is_available() else (lambda: None)
    except Exception:  # torch is plumbing only
        sync = lambda: None  # noqa: E731

    instances = WORKLOADS[args.workload]
    want = expected_values()
    if args.workload == "pt":
        learned_cfg = dict(hidden1=256, hidden2=256, first_level=args.pt_learned_first,
                           plain_per_learned=args.pt_learned_every, snapshots=8, train_steps=400, minibatch=1024,
                           lr=1e-3, init_seed=1)
        sync()
        t0 = time.perf_counter()
        pt = pt_bench(sk, want, [1 << int(x) for x in args.pt_plain_log2.split(",")],
                      [1 << int(x) for x in args.pt_learned_log2.split(",") if x],
                      [1 << int(x) for x in args.pt_tuned_log2.split(",") if x], args.pt_ladders, learned_cfg,
                      cpu_pt=not args.no_cpu_baseline)
        sync()
        elapsed = time.perf_counter() - t0
        plain = [r for r in pt["runs"] if r["proposal"] == "plain"]
        moves = sum(r["level_moves"] for r in plain)
        gpu_s = sum(r["gpu_s"] for r in plain)
        print(json.dumps({"metric": METRIC, "value": moves / gpu_s, "unit": "level-moves/s", "n_gpus": 1,
                          "steps": 1, "warmup": 0, "ms_per_step": elapsed * 1e3, "higher_is_better": True,
                          "scaling": "weak", "vs_baseline": None, "dtype": "u32", "data": "synthetic",
                          "config": {"workload": "pt", "ladders": args.pt_ladders, "levels": pt["levels"]},
                          "pt": pt}), flush=True)
        return
    tuning = {"log2_chunk_terms": args.log2_chunk, "kernel": args.kernel, "waves_per_launch": args.waves}
    if args.workload == "s12":
        tuning["primes"] = 2
    batched = args.workload in ("batch", "mixed", "all24") and not args.separate

    slice_ids = None
    if args.workload == "l28slice":
        from paper_1507_00315_amd import inputs
        slice_ids = inputs.distinct_ids(inputs.SLICE_SEED, L28_CHUNK_BITS, L28_SLICE)
        slice_primes = sk.describe(28, "langford")["primes"]  # default primes, as a full count uses
    n24 = n24_slices() if args.workload == "mixed" else []
    # device workspaces owned by torch, so that a timed step allocates nothing
    ws_count = ws_slice = None
    if batched:
        import torch
        ws_count = torch.empty(sk.workspace_bytes([(n, v) for v, n in instances]), dtype=torch.uint8,
                               device="cuda")
        if n24:
            ws_slice = torch.empty(max(sk.partial_workspace_bytes(24, sl["variant"], len(sl["ids"]),
                                                                  len(sl["primes"])) for sl in n24),
                                   dtype=torch.uint8, device="cuda")

    def run_slice(tag, sl):
        """One n = 24 slice: 8192 chunks in one call; the rows the oracle
        recomputed must match."""
        rows, st = sk.partial_chunks(24, sl["variant"], sl["log2_chunks"], sl["ids"], sl["primes"], with_stats=True,
                                     workspace=ws_slice)
        ok = all(rows[i] == want_row for i, want_row in sl["check"])
        log(f"[{tag}] {sl['variant']} n=24 slice: kernel {st['kernel_ms']:.1f} ms "
            f"{st['terms'] / max(st['kernel_ms'], 1e-9) * 1e3:.3e} terms/s  check={ok}")
        return (sl["variant"], 24, None, st, ok)

    def step(tag):
        res = []
        if slice_ids is not None:
            t0 = time.time()
            rows, st = sk.partial_chunks(28, "langford", L28_CHUNK_BITS, slice_ids, slice_primes,
                                         tuning=tuning if args.log2_chunk or args.kernel else None,
                                         with_stats=True)
            res.append(("langford", 28, None, st, None))
            log(f"[{tag}] l28 slice: {len(rows)} chunks, kernel {st['kernel_ms']:.1f} ms "
                f"{st['terms'] / max(st['kernel_ms'], 1e-9) * 1e3:.3e} terms/s  wall {time.time() - t0:.1f} s")
            return res
        if batched:
            counts, st = sk.count_batch([(n, v, sk.ORDERED if v == "hooked" else 0) for v, n in instances],
                                        tuning=tuning if args.log2_chunk else None, workspace=ws_count)
            checks = []
            for (v, n), c in zip(instances, counts):
                ok = want.get((v, n))
                checks.append(None if ok is None else (ok == c))
            res.append(("*", 0, counts, st, all(x is not False for x in checks)))
            log(f"[{tag}] batch: kernel {st['kernel_ms']:.1f} ms  {st['terms'] / max(st['kernel_ms'], 1e-9) * 1e3:.3e}"
                f" terms/s  launches {st['launches']}  checks {checks}")
            for sl in n24:
                res.append(run_slice(tag, sl))
            return res
        last = [time.time()]

        def progress(done, total):
            if time.time() - last[0] > 20:
                last[0] = time.time()
                log(f"  ... {done / total * 100:.1f}% of {total:.3e} sign vectors")
            return False

        for v, n in instances:
            if args.workload.startswith("larsen"):
                r = sk.count_larsen(n, v, ordered=(v == "hooked"), tuning=tuning)
            else:
                r = sk.count_ex(n, v, ordered=(v == "hooked"), tuning=tuning, progress=progress)
            ok = want.get((v, n))
            res.append((v, n, r.count, r.stats, None if ok is None else (ok == r.count)))
            log(f"[{tag}] {v} n={n}: {r.count}  kernel {r.stats['kernel_ms']:.1f} ms  "
                f"{r.stats['terms'] / max(r.stats['kernel_ms'], 1e-9) * 1e3:.3e} terms/s  "
                f"check={res[-1][4]}")
        return res

    launch_waves = args.waves
    if args.workload in ("batch", "mixed") and batched and not args.no_autotune and not args.log2_chunk:
        t0 = time.time()
        best, rate = sk.autotune_batch([(n, v) for v, n in instances])
        launch_waves = best["waves_per_launch"]
        log(f"autotune: {best} ({rate:.3e} terms/s on the probe, {time.time() - t0:.1f} s)")
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

    # Per kernel: VALU instructions per sign vector (design count of the tuned
    # body) x sign vectors / launch durations measured with HIP events on the
    # launch stream.
    def design_instr(v, n, symmetric_terms):
        d = sk.describe(n, v)
        d["primes_used"] = d["primes"]
        per = valu_per_term(d)
        if symmetric_terms:
            r = d["reversal_quads"] if results[0][0][3]["reversal_quads"] else 0
            terms = ((1 << (2 * n - 1)) >> d["symmetric"]) // 2 ** (r + 1) * (2 ** r + 1)
        else:
            terms = None
        return per, terms, ring_ops_per_term(n, d["primes"])

    # (name, kernel, terms per step, VALU instr per step, ring ops per step,
    #  results index, key of the measured traffic or None)
    legs = []
    if slice_ids is not None:
        per, _, ring = design_instr("langford", 28, False)
        legs.append(("langford:28 slice", sk.kernel_name(results[0][0][3]["kernel_variant"]), terms_per_step,
                     per * terms_per_step, ring * terms_per_step, 0, None))
    elif batched:
        instr = ring = 0
        for v, n in instances:
            per, terms, rg = design_instr(v, n, True)
            instr += per * terms
            ring += rg * terms
        legs.append(("batch", "exact_batch_kernel", results[0][0][3]["terms"], instr, ring, 0,
                     ("exact_batch_kernel", "batch" if args.workload == "mixed" else args.workload,
                      results[0][0][3]["log2_chunk_terms"], launch_waves)))
        for i, sl in enumerate(n24):
            per, _, rg = design_instr(sl["variant"], 24, False)
            t = results[0][1 + i][3]["terms"]
            legs.append((f"{sl['variant']}:24 slice", f"exact_v2_kernel<{sk.VARIANTS[sl['variant']]},24>", t,
                         per * t, rg * t, 1 + i,
                         ("exact_v2_kernel", f"{sl['variant']}:24 slice", results[0][1 + i][3]["log2_chunk_terms"],
                          len(sl["ids"]))))
    elif args.workload.startswith("larsen"):
        for i, (v, n) in enumerate(instances):
            d = sk.describe(n, v, larsen=True)
            d["primes_used"] = d["primes"]
            t = results[0][i][3]["terms"]
            legs.append((f"{v}:{n} inclusion-exclusion", sk.kernel_name(results[0][i][3]["kernel_variant"]), t,
                         valu_per_term(d) * t, ring_ops_per_term(n, d["primes"]) * t, i, None))
    else:
        for i, (v, n) in enumerate(instances):
            per, terms, rg = design_instr(v, n, True)
            t = results[0][i][3]["terms"]
            legs.append((f"{v}:{n}", sk.kernel_name(results[0][i][3]["kernel_variant"]), t, per * t, rg * t, i,
                         None))

    rooflines = []
    for name, kernel, terms, instr, ring, idx, tkey in legs:
        kms = sum(st[idx][3]["kernel_ms"] for st in results) / args.steps
        launches = sum(st[idx][3]["launches"] for st in results) // args.steps
        sec = kms * 1e-3
        rooflines.append({"leg": name, "kernel": kernel, "bound": "alu", "unit": "VALU lane-instr/s",
                          "achieved": instr / sec if sec > 0 else 0.0, "peak": PEAK_LANE_OPS,
                          "frac": instr / sec / PEAK_LANE_OPS if sec > 0 else 0.0,
                          "valu_instr_per_term": instr / terms, "terms_per_launch_step": terms,
                          "terms_per_s_kernel": terms / sec if sec > 0 else 0.0, "kernel_ms_per_step": kms,
                          "launches": launches, "avg_launch_ms": kms / max(launches, 1),
                          "ring_ops_per_term": ring / terms,
                          "traffic": traffic_per_launch(*tkey) if tkey else None})
    # the dominant kernel: the single kernel with the largest time per step
    dom = max(rooflines, key=lambda r: r["avg_launch_ms"])
    st0 = results[0][0][3]
    log2_chunk = st0["log2_chunk_terms"]
    roofline = {"bound": "alu", "achieved": dom["achieved"], "peak": PEAK_LANE_OPS, "unit": "VALU lane-instr/s",
                "frac": dom["frac"], "traffic": dom["traffic"],
                "kernel": dom["kernel"], "leg": dom["leg"], "valu_instr_per_term": dom["valu_instr_per_term"],
                "terms_per_s_kernel": dom["terms_per_s_kernel"], "launches": dom["launches"],
                "avg_launch_ms": dom["avg_launch_ms"],
                "note": "achieved = design VALU instructions per sign vector x sign vectors / kernel time; the "
                        "method's ring-operation count per term (ring_ops_per_term) is not an issue roof: "
                        "packed 16-bit adds, scalar-unit pair-sum updates and products shared across primes "
                        "do several ring operations per VALU lane-instruction"}

    covered = 0
    if slice_ids is not None:
        covered = terms_per_step
    elif batched:
        covered = sum(1 << (2 * n - 1) for v, n in instances) + sum(results[0][1 + i][3]["terms"]
                                                                     for i in range(len(n24)))
    elif args.workload.startswith("larsen"):
        covered = terms_per_step
    else:
        covered = sum(1 << (2 * n - 1) for v, n in instances)
    config = {"workload": args.workload,
              "instances": [f"{v}:{n}" for v, n in instances],
              "terms_per_step": terms_per_step,
              "primes_per_instance": {f"{v}:{n}": sk.describe(n, v)["primes"] for v, n in instances},
              "log2_chunk_terms": log2_chunk,
              "waves_per_launch": launch_waves,
              "lemma_2_4_halving": bool(st0.get("symmetry_halved")),
              "sign_vectors_covered_per_step": covered,
              "sign_vectors_covered_per_s": covered * args.steps / elapsed,
              "reversal_quads": st0.get("reversal_quads", 0),
              "results_match_expected": all_ok}
    if n24:
        config["n24_slices"] = [{"instance": f"{sl['variant']}:24", "chunks": len(sl["ids"]),
                                 "of_chunks": 1 << sl["log2_chunks"],
                                 "sign_vectors_per_chunk": 1 << (47 - sl["log2_chunks"]), "seed": sl["seed"],
                                 "primes": len(sl["primes"]), "rows_checked_per_step": len(sl["check"])}
                                for sl in n24]
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
        "config": config,
        "roofline": roofline,
        "rooflines": rooflines,
    }
    if slice_ids is not None:
        full_chunks = 1 << L28_CHUNK_BITS
        kms = rooflines[0]["kernel_ms_per_step"]
        line["config"]["slice"] = {"chunks": len(slice_ids), "of_chunks": full_chunks,
                                   "terms_per_chunk": terms_per_step // len(slice_ids), "seed": 1507,
                                   "projected_full_count_s": kms * 1e-3 * full_chunks / len(slice_ids),
                                   "projected_full_count_wall_s": elapsed / args.steps * full_chunks / len(slice_ids)}
    if args.workload in ("batch", "mixed") and batched and not args.no_pt:
        learned_cfg = dict(hidden1=256, hidden2=256, first_level=args.pt_learned_first,
                           plain_per_learned=args.pt_learned_every, snapshots=8, train_steps=400, minibatch=1024,
                           lr=1e-3, init_seed=1)
        line["pt"] = pt_bench(sk, want, [1 << int(x) for x in args.pt_plain_log2.split(",")],
                              [1 << int(x) for x in args.pt_learned_log2.split(",") if x],
                              [1 << int(x) for x in args.pt_tuned_log2.split(",") if x], args.pt_ladders,
                              learned_cfg, cpu_pt=not args.no_cpu_baseline)
    if not args.no_cpu_baseline:
        log("cpu baseline ...")
        line["cpu_baseline"] = cpu_baseline(instances)
    print(json.dumps(line), flush=True)
    if not all_ok:
        sys.exit(1)


if __name__ == "__main__":
    main()
