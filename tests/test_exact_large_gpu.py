"""GPU parity of the exact path at n = 22..25 (the configurations the
benchmark's n = 24 figures and the largest single-GPU counts come from).

* L(23), S(24) and L(24) as full counts against the printed values (Table 4,
  Tables 7 and 8), reported and ordered; with every count n <= 21 checked in
  tests/test_exact_gpu.py this covers every nonzero S(n), L(n) with n <= 24.
* S(22) and L(22) with the existence shortcut off: the evaluated sum must
  vanish (Sec. 1.1).
* Per-chunk residues of S(24), L(24) (2^26 sign vectors per chunk, in the
  8192-chunk launch the benchmark times) and S(25) (2^28 per chunk, the n = 25
  kernel) against the oracle's recomputation stored by
  tests/golden/make_big_chunks.py.
* Single jobs of S(24) and L(24) whose products leave the two-group chain's
  exact range (the kernel evaluates them again with three groups) against the
  oracle computed in the test; chunks of L(30) with ids of 33 bits (four
  product groups) likewise.
"""
import json
import os
import sys

import pytest

import oracle as O
import paper_1507_00315_amd as sk
from paper_1507_00315_amd import inputs

pytestmark = pytest.mark.gpu

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _load(name):
    with open(os.path.join(GOLD, name)) as f:
        return json.load(f)


def _say(*a):
    print(*a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module", autouse=True)
def _ready():
    sk.lib()


def test_printed_counts_n23_n24():
    """L(23), S(24), L(24) as full exact counts with both symmetries (Lemma
    2.3, Lemma 2.4) in one persistent launch (their batched group), against
    the printed values (Tables 7 and 8); the ordered counts are twice the
    printed ones (Sec. 1.3) and equal Table 4's for S(24)."""
    paper = _load("paper_counts.json")
    inst = [(23, "langford", sk.ORDERED), (24, "skolem", sk.ORDERED), (24, "langford", sk.ORDERED)]
    _say("full counts L(23), S(24), L(24) in one batched launch")
    counts, st = sk.count_batch(inst, tuning={"log2_chunk_terms": 30, "waves_per_launch": 8192})
    _say(f"  {counts}  kernel {st['kernel_ms'] / 1e3:.1f} s, launches {st['launches']}")
    assert st["launches"] == 1 and st["kernel_variant"] == 3
    for (n, v, _), c in zip(inst, counts):
        assert c == 2 * int(paper[v][str(n)]), (v, n)
    assert counts[1] == int(paper["skolem_ordered"]["24"])


@pytest.mark.parametrize("variant", ["skolem", "langford"])
def test_nonexistent_n22_sum_vanishes(variant):
    """n = 22 has no Skolem (n = 2 mod 4) and no Langford (n = 2 mod 4)
    pairing; with the shortcut off the whole signed sum is evaluated."""
    _say("zero", variant, 22)
    r = sk.count_ex(22, variant, ordered=True, no_shortcut=True)
    assert r.count == 0
    assert r.stats["terms"] > 0 and r.stats["symmetry_halved"] == 0


def _case(key):
    g = _load("big_chunks.json")
    return g["primes"], g["cases"][key]


@pytest.mark.parametrize("variant", ["skolem", "langford"])
def test_n24_slice_chunks_match_oracle(variant):
    """The benchmark's n = 24 slice: 8192 chunks of 2^26 sign vectors in one
    call, in its launch shape; the 16 chunks the oracle recomputed must match
    bit for bit, and repeating the call gives the same rows."""
    primes, c = _case(f"{variant}:24")
    ids = inputs.distinct_ids(c["slice_seed"], c["log2_chunks"], c["slice_size"])
    assert c["slice_size"] == inputs.N24_SLICE and c["log2_chunks"] == inputs.N24_CHUNK_BITS
    rows, st = sk.partial_chunks(24, variant, c["log2_chunks"], ids, primes, with_stats=True)
    _say(f"{variant} 24 slice: {st['kernel_ms']:.1f} ms, body {st['kernel_variant']}")
    assert st["kernel_variant"] == 2 and st["terms"] == len(ids) << 26
    pos = {cid: i for i, cid in enumerate(ids)}
    for ch in c["chunks"]:
        assert rows[pos[ch["id"]]] == [int(x) for x in ch["residues"]], ch["id"]
    again = sk.partial_chunks(24, variant, c["log2_chunks"], ids, primes)
    assert again == rows


def test_s25_chunks_match_oracle():
    """The n = 25 kernel (two primes cover 25!; Sec. 2.2's split into
    independent parts) on 8 chunks of 2^28 sign vectors."""
    primes, c = _case("skolem:25")
    ids = [ch["id"] for ch in c["chunks"]]
    assert ids == inputs.distinct_ids(inputs.S25_SEED, inputs.S25_CHUNK_BITS, inputs.S25_CHUNKS)
    rows, st = sk.partial_chunks(25, "skolem", c["log2_chunks"], ids, primes, with_stats=True)
    assert st["kernel_variant"] == 2
    for ch, row in zip(c["chunks"], rows):
        assert row == [int(x) for x in ch["residues"]], ch["id"]
    ref = sk.partial_chunks(25, "skolem", c["log2_chunks"], ids[:2], primes, tuning={"kernel": 1})
    assert ref == rows[:2]


def _product_at_all_plus(n, variant):
    """|prod_k f_k| (factors with an even pair count halved, as the kernel
    holds them) at x = +1...+1, where f_k is the number of pairs at d_k."""
    pos, d = O.instance(n, variant)
    ps = set(pos)
    prod = 1
    for dk in d:
        L = sum(1 for p in pos if p + dk in ps)
        prod *= L // 2 if L % 2 == 0 else L
    return prod


@pytest.mark.parametrize("variant,n", [("skolem", 24), ("langford", 24), ("hooked", 23)])
def test_jobs_outside_the_fast_chain_match_oracle(variant, n):
    """Chunks of one job each (chunk bits = every job variable).  Three jobs
    hold nearly periodic sign vectors whose products exceed 2^96, beyond the
    two-group chain, so the kernel must redo the segments that hold them with
    the full chain: every job variable +1 (x = +1...+1 lies in it), the job
    variables alternating as in x_p = (-1)^(p+1) (the alternating vector), and
    every job variable -1.  Three seeded ids are ordinary jobs.  Every row must
    equal the oracle's Gray-walk sum over the same sign vectors."""
    assert _product_at_all_plus(n, variant) >= 1 << 96  # |f_k| = L_k at both patterns
    c = sk.max_chunk_bits(n, variant)
    pos, _ = O.instance(n, variant)
    m = len(pos)
    job_pos = [pos[m - 6 - c + b] for b in range(c)]
    alternating = sum(1 << b for b, p in enumerate(job_pos) if p % 2 == 0)
    ids = [0, alternating, (1 << c) - 1] + inputs.distinct_ids(2424, c, 3)
    primes = O.primes_below(1 << 46, 2)
    _say(f"{variant} {n}: {len(ids)} single-job chunks of {c} chunk bits")
    rows = sk.partial_chunks(n, variant, c, ids, primes)
    for cid, row in zip(ids, rows):
        fixed = {pos[0]: 1}
        for b in range(c):
            fixed[job_pos[b]] = -1 if (cid >> b) & 1 else 1
        want = [O.chunk_partial(n, variant, fixed, p, "gray", threads=8) for p in primes]
        assert row == want, (variant, n, hex(cid))


def test_chunk_ids_above_32_bits_match_oracle():
    """Langford n = 30 with its 33 chunk variables (chunks of 2^26 sign
    vectors): chunk ids with bit 31 and bit 32 set (the wave reads an id as two
    32-bit halves), four product groups merged into two by the fast chain.
    Ids: every chunk variable -1 (products near the maximum, reached in a
    segment in the middle of the walk), bit 31 alone, the alternating
    pattern, and two seeded ids with bit 32 set."""
    n, variant, c = 30, "langford", 33
    assert sk.max_chunk_bits(n, variant) == c
    ids = [(1 << c) - 1, 1 << 31, 0x155555555] + [x | (1 << 32) for x in inputs.distinct_ids(3030, 31, 2)]
    primes = O.primes_below(1 << 46, 3)
    _say(f"{variant} {n}: {len(ids)} chunks of 2^26 sign vectors, ids up to 33 bits")
    rows = sk.partial_chunks(n, variant, c, ids, primes)
    pos, _ = O.instance(n, variant)
    m = len(pos)
    for cid, row in zip(ids, rows):
        fixed = {pos[0]: 1}
        for b in range(c):
            fixed[pos[m - 6 - c + b]] = -1 if (cid >> b) & 1 else 1
        want = [O.chunk_partial(n, variant, fixed, p, "gray", threads=8) for p in primes]
        assert row == want, (variant, n, hex(cid))
