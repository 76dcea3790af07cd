"""Writes tests/golden/big_chunks.json: partial sums of chunks of the n = 24
and n = 25 sign-vector sums (Lemma 2.1), recomputed on the CPU by the
oracle's Gray-code walk modulo the primes a full count uses (the two largest
primes below 2^46).

* Skolem n = 24 and Langford n = 24: 16 chunks of 2^26 sign vectors each,
  picked (seed + 1) from the 8192-chunk slices the benchmark times (seeds in
  paper_1507_00315_amd/inputs.py);
* Skolem n = 25: 8 chunks of 2^28 sign vectors each.

The chunk definition (which sign variables a chunk id fixes) is the one
documented for sk_partial_chunks in include/skolem.h.  Calls only ``oracle``
and the seeded input module.

    python tests/golden/make_big_chunks.py [threads]
"""
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)
import oracle as O  # noqa: E402
from paper_1507_00315_amd import inputs  # noqa: E402  (seeded generators only)

HERE = os.path.dirname(os.path.abspath(__file__))
OUT = os.path.join(HERE, "big_chunks.json")


def chunk_fixed(n, variant, c, cid):
    pos, _ = O.instance(n, variant)
    m = len(pos)
    fixed = {pos[0]: 1}
    for b in range(c):
        rank = m - 6 - c + 1 + b
        fixed[pos[rank - 1]] = -1 if (cid >> b) & 1 else 1
    return fixed


def cases():
    for v in ("skolem", "langford"):
        seed = inputs.N24_SLICE_SEEDS[v]
        ids = inputs.distinct_ids(seed, inputs.N24_CHUNK_BITS, inputs.N24_SLICE)
        yield {"key": f"{v}:24", "n": 24, "variant": v, "log2_chunks": inputs.N24_CHUNK_BITS,
               "slice_seed": seed, "slice_size": inputs.N24_SLICE, "pick_seed": seed + 1,
               "ids": inputs.subset(seed + 1, ids, 16)}
    yield {"key": "skolem:25", "n": 25, "variant": "skolem", "log2_chunks": inputs.S25_CHUNK_BITS,
           "slice_seed": inputs.S25_SEED, "slice_size": inputs.S25_CHUNKS,
           "ids": inputs.distinct_ids(inputs.S25_SEED, inputs.S25_CHUNK_BITS, inputs.S25_CHUNKS)}


def main():
    threads = int(sys.argv[1]) if len(sys.argv) > 1 else (os.cpu_count() or 1)
    O.build(force=False)
    primes = O.primes_below(1 << 46, 2)
    out = {"_source": "oracle.chunk_partial (Gray-code walk), written by make_big_chunks.py",
           "primes": primes, "cases": {}}
    if os.path.exists(OUT):
        with open(OUT) as f:
            prev = json.load(f)
        if prev.get("primes") == primes:
            out["cases"] = prev.get("cases", {})
    for c in cases():
        have = {ch["id"]: ch for ch in out["cases"].get(c["key"], {}).get("chunks", [])}
        rec = {k: v for k, v in c.items() if k not in ("key", "ids")}
        rec["chunks"] = []
        for cid in c["ids"]:
            if cid in have:
                rec["chunks"].append(have[cid])
                continue
            t0 = time.time()
            res = [O.chunk_partial(c["n"], c["variant"], chunk_fixed(c["n"], c["variant"], c["log2_chunks"], cid),
                                   p, "gray", threads=threads) for p in primes]
            rec["chunks"].append({"id": cid, "residues": res, "seconds": round(time.time() - t0, 1)})
            print(c["key"], cid, res, f"{time.time() - t0:.1f}s", flush=True)
            out["cases"][c["key"]] = rec
            with open(OUT, "w") as f:
                json.dump(out, f, indent=1)
        out["cases"][c["key"]] = rec
    with open(OUT, "w") as f:
        json.dump(out, f, indent=1)


if __name__ == "__main__":
    main()
