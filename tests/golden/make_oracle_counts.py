"""Writes tests/golden/oracle_counts.json: ordered counts from the CPU oracle's
backtracking search for instances too slow to search inside the test suite.

Calls only ``oracle``.  Where the paper prints a value (Tables 7 and 8) the
script checks the oracle against it before writing.

    python tests/golden/make_oracle_counts.py [threads]
"""
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)
import oracle as O  # noqa: E402

HERE = os.path.dirname(os.path.abspath(__file__))
OUT = os.path.join(HERE, "oracle_counts.json")

JOBS = [("hooked", n) for n in range(1, 16)] + [("skolem", 16), ("langford", 15), ("langford", 16)]


def main():
    threads = int(sys.argv[1]) if len(sys.argv) > 1 else os.cpu_count()
    O.build(force=False)
    with open(os.path.join(HERE, "paper_counts.json")) as f:
        paper = json.load(f)
    out = {}
    if os.path.exists(OUT):
        with open(OUT) as f:
            out = json.load(f)
    out["_source"] = ("ordered counts (reflections distinct) from oracle.count_backtrack; "
                      "written by tests/golden/make_oracle_counts.py")
    for variant, n in JOBS:
        key = f"{variant}:{n}"
        if key in out:
            continue
        t0 = time.time()
        c = O.count_backtrack(n, variant, threads=threads)
        dt = time.time() - t0
        printed = paper.get(variant, {}).get(str(n))
        if printed is not None:
            assert O.reported(c, n, variant) == int(printed), (variant, n, c, printed)
        out[key] = {"ordered": str(c), "seconds": round(dt, 2), "threads": threads,
                    "matches_paper": printed is not None}
        print(key, c, f"{dt:.1f}s", flush=True)
        with open(OUT, "w") as f:
            json.dump(out, f, indent=1, sort_keys=True)


if __name__ == "__main__":
    main()
