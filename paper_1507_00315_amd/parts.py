"""Run one exact count as independent parts and put it together (Sec. 2.2).

    python -m paper_1507_00315_amd.parts run --n 27 --variant langford --parts 8 --part 0 --part 1 --out DIR
    python -m paper_1507_00315_amd.parts combine --n 27 --variant langford --parts 8 DIR

`run` evaluates the listed parts on this GPU and writes one JSON file per part
(its residues modulo the count's primes, and the launch statistics); the parts
can run in different processes, on different GPUs or machines.  `combine`
(host only) reads every part's file and prints the count.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

from . import count_combine, count_part, describe


def _path(out: str, variant: str, n: int, part: int, parts: int) -> str:
    return os.path.join(out, f"{variant}{n}_part{part}of{parts}.json")


def run(n: int, variant: str, parts: int, which, out: str, ordered: bool) -> None:
    os.makedirs(out, exist_ok=True)
    for part in which:
        t0 = time.time()
        last = [t0]

        def progress(done, total):
            if time.time() - last[0] > 20:
                last[0] = time.time()
                print(f"  part {part}: {done / total * 100:.1f}% of {total:.3e} sign vectors", flush=True)
            return False

        residues, st = count_part(n, variant, part, parts, ordered=ordered, progress=progress)
        rec = {"n": n, "variant": variant, "ordered": ordered, "part": part, "parts": parts,
               "residues": residues, "primes": st["primes"], "kernel_ms": st["kernel_ms"],
               "terms": st["terms"], "wall_s": time.time() - t0}
        with open(_path(out, variant, n, part, parts), "w") as f:
            json.dump(rec, f)
        print(f"part {part}/{parts}: kernel {st['kernel_ms'] / 1e3:.1f} s, "
              f"{st['terms'] / max(st['kernel_ms'], 1e-9) * 1e3:.3e} terms/s", flush=True)


def combine(n: int, variant: str, parts: int, src: str, ordered: bool) -> int:
    rows = []
    kernel_s = 0.0
    for part in range(parts):
        p = _path(src, variant, n, part, parts)
        if not os.path.exists(p):
            raise SystemExit(f"missing part {part}: {p}")
        with open(p) as f:
            rec = json.load(f)
        if (rec["n"], rec["variant"], rec["parts"], rec["ordered"]) != (n, variant, parts, ordered):
            raise SystemExit(f"{p} belongs to another run")
        rows.append(rec["residues"])
        kernel_s += rec["kernel_ms"] / 1e3
    c = count_combine(n, variant, rows, ordered=ordered)
    print(json.dumps({"n": n, "variant": variant, "ordered": ordered, "count": str(c), "parts": parts,
                      "kernel_s_total": kernel_s, "primes": describe(n, variant)["primes"]}))
    return c


def main(argv=None) -> None:
    ap = argparse.ArgumentParser(prog="python -m paper_1507_00315_amd.parts")
    sub = ap.add_subparsers(dest="cmd", required=True)
    r = sub.add_parser("run")
    c = sub.add_parser("combine")
    for p in (r, c):
        p.add_argument("--n", type=int, required=True)
        p.add_argument("--variant", default="skolem", choices=["skolem", "langford", "hooked"])
        p.add_argument("--parts", type=int, required=True)
        p.add_argument("--ordered", action="store_true")
    r.add_argument("--part", type=int, action="append", required=True)
    r.add_argument("--out", required=True)
    c.add_argument("src")
    a = ap.parse_args(argv)
    if a.cmd == "run":
        run(a.n, a.variant, a.parts, a.part, a.out, a.ordered)
    else:
        combine(a.n, a.variant, a.parts, a.src, a.ordered)


if __name__ == "__main__":
    main(sys.argv[1:])
