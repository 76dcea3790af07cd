"""GPU parity of the exact path against the CPU oracle (bit-exact).

Runs through the C ABI (paper_1507_00315_amd binding).  Expected values come
from the oracle (computed here, or stored by tests/golden/make_oracle_counts.py)
or from the paper's printed tables (tests/golden/paper_counts.json).
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
    O.build(force=False)
    sk.lib()


# Moduli for residue comparisons: chosen by the oracle's own prime search.
PRIMES = O.primes_below(1 << 46, 8)


@pytest.mark.parametrize("variant", ["skolem", "langford", "hooked"])
def test_counts_small_n_all_variants(variant):
    """Ordered counts for n = 1..12 with the existence shortcut disabled, so
    the sum is evaluated (and must vanish) where no pairing exists."""
    for n in range(1, 13):
        _say("count", variant, n)
        want = O.count_backtrack(n, variant, threads=8)
        got = sk.count(n, variant, ordered=True, no_shortcut=True)
        assert got == want, (variant, n, got, want)


def test_reported_counts_at_n1():
    """S(1) = 1: the one pairing is its own reflection and is not halved
    (Sec. 1.3 halves for n > 1); L(1) = 0; the sum is evaluated."""
    assert sk.count(1, "skolem", no_shortcut=True) == 1
    assert sk.count(1, "skolem", ordered=True, no_shortcut=True) == 1
    assert sk.count(1, "langford", no_shortcut=True) == 0
    assert sk.count_larsen(1, "skolem", no_shortcut=True).count == 1


def test_skolem_12_without_symmetries_and_zeros():
    """S(12) over 2^23 sign vectors, two primes; S(10) = S(11) = 0 (Table 7;
    existence, Sec. 1.1)."""
    r = sk.count_ex(12, "skolem", tuning={"primes": 2}, no_symmetry=True)
    assert r.count == 227968
    assert r.stats["nprimes"] == 2 and r.stats["terms"] == 1 << 23 and r.stats["symmetry_halved"] == 0
    # by default only the Lemma 2.4 half is evaluated, of which the reversal
    # weights (Lemma 2.3) keep 1/2 + 2^-(r+1)
    h = sk.count_ex(12, "skolem", tuning={"primes": 2})
    r = h.stats["reversal_quads"]
    assert h.count == 227968 and h.stats["symmetry_halved"] == 1 and r >= 1
    assert h.stats["terms"] == (1 << 22) // 2 ** (r + 1) * (2 ** r + 1)
    for n in (10, 11):
        assert sk.count(n, "skolem", no_shortcut=True) == 0
    assert O.is_valid_pairing(O.skolem_construction(12), 12, "skolem")


@pytest.mark.parametrize("variant", ["skolem", "langford", "hooked"])
def test_sign_sum_residues_match_oracle(variant):
    for n in (5, 8, 9, 11, 12):
        _say("residues", variant, n)
        primes = PRIMES[3:6]
        got = sk.sign_sum_residues(n, variant, primes)
        want = [O.chunk_partial(n, variant, {1: 1}, p, "gray", threads=8) for p in primes]
        assert got == want, (variant, n)


@pytest.mark.parametrize("variant", ["skolem", "langford", "hooked"])
@pytest.mark.parametrize("kernel", [1, 2])
def test_both_kernel_bodies_match_oracle(variant, kernel):
    """The reference body (1) and the tuned body (2) against the oracle, on the
    smallest instances the tuned body is built for (several unrolled blocks,
    several jobs per chunk, every outer walked variable flipped)."""
    for n in (13, 14):
        _say("kernel", kernel, variant, n)
        primes = PRIMES[:3]
        got = sk.sign_sum_residues(n, variant, primes, tuning={"kernel": kernel})
        want = [O.chunk_partial(n, variant, {1: 1}, p, "gray", threads=8) for p in primes]
        assert got == want, (variant, n, kernel)


@pytest.mark.parametrize("variant,n", [("skolem", 16), ("langford", 16), ("hooked", 15), ("skolem", 20),
                                       ("langford", 19), ("skolem", 24)])
def test_tuned_body_equals_reference_body_on_chunks(variant, n):
    """Per-chunk residues of the two kernel bodies agree bit for bit (chunks
    drawn with a seeded stream; the oracle checks the small sizes above)."""
    c = sk.max_chunk_bits(n, variant)
    ids = inputs.distinct_ids(1000 + n, c, 64)
    primes = PRIMES[:2]
    a = sk.partial_chunks(n, variant, c, ids, primes, tuning={"kernel": 1})
    b = sk.partial_chunks(n, variant, c, ids, primes, tuning={"kernel": 2})
    assert a == b


def _chunk_fixed(n, variant, c, cid):
    """Fixed assignment of a chunk, from the chunk definition in skolem.h."""
    pos, _ = O.instance(n, variant)
    m = len(pos)
    fixed = {pos[0]: 1}
    for b in range(c):
        rank = m - 6 - c + 1 + b
        fixed[pos[rank - 1]] = -1 if (cid >> b) & 1 else 1
    return fixed


@pytest.mark.parametrize("kernel", [1, 2])
@pytest.mark.parametrize("variant,n", [("skolem", 12), ("langford", 13), ("hooked", 12), ("skolem", 13)])
def test_partial_chunks_match_oracle(variant, n, kernel):
    cmax = sk.max_chunk_bits(n, variant)
    c = min(cmax, 6)
    ids = inputs.distinct_ids(42 + n, c, min(8, 1 << c))
    primes = PRIMES[:2]
    got = sk.partial_chunks(n, variant, c, ids, primes, tuning={"kernel": kernel})
    for cid, row in zip(ids, got):
        fixed = _chunk_fixed(n, variant, c, cid)
        want = [O.chunk_partial(n, variant, fixed, p, "gray", threads=8) for p in primes]
        assert row == want, (variant, n, cid)


def test_chunk_partials_sum_to_total():
    n, v = 13, "skolem"
    c = sk.max_chunk_bits(n, v)
    primes = PRIMES[:3]
    rows = sk.partial_chunks(n, v, c, list(range(1 << c)), primes)
    tot = sk.sign_sum_residues(n, v, primes)
    for i, p in enumerate(primes):
        assert sum(r[i] for r in rows) % p == tot[i]


@pytest.mark.parametrize("log2_chunk", [17, 20, 23, 26, 31])
def test_launch_shape_does_not_change_result(log2_chunk):
    r = sk.count_ex(13, "skolem", tuning={"log2_chunk_terms": log2_chunk, "waves_per_launch": 64})
    assert r.count == 1520280
    assert r.stats["kernel_variant"] == 2


def test_repeat_runs_bit_identical():
    a = sk.sign_sum_residues(14, "langford", PRIMES[:4])
    b = sk.sign_sum_residues(14, "langford", PRIMES[:4])
    assert a == b


def test_verify_flag_two_disjoint_prime_sets():
    r = sk.count_ex(13, "skolem", verify=True)
    assert r.count == 1520280 and r.stats["passes"] == 2
    assert len(set(r.stats["primes"])) == 2 * r.stats["nprimes"]


@pytest.mark.parametrize("variant,n", [("skolem", 16), ("skolem", 17), ("langford", 15), ("langford", 16)])
def test_printed_values_mid(variant, n):
    want = int(_load("paper_counts.json")[variant][str(n)])
    _say("printed", variant, n)
    assert sk.count(n, variant) == want


@pytest.mark.parametrize("n", [13, 14, 15])
def test_hooked_against_stored_oracle(n):
    g = _load("oracle_counts.json")
    want = int(g[f"hooked:{n}"]["ordered"])
    assert sk.count(n, "hooked", no_shortcut=True) == want


def test_small_instances_use_reference_body():
    r = sk.count_ex(9, "skolem", no_shortcut=True)
    assert r.count == 1328 and r.stats["kernel_variant"] == 1


def test_invalid_arguments():
    with pytest.raises(sk.SkolemError):
        sk.count(0, "skolem")
    with pytest.raises(sk.SkolemError):
        sk.count(33, "skolem")
    with pytest.raises(sk.SkolemError):
        sk.partial_chunks(12, "skolem", 99, [0], PRIMES[:1])
    with pytest.raises(sk.SkolemError):
        sk.partial_chunks(12, "skolem", 2, [4], PRIMES[:1])  # id >= 2^c
    with pytest.raises(sk.SkolemError):
        sk.sign_sum_residues(8, "skolem", [1000003])  # prime below the supported range


MIXED = [(16, "skolem"), (17, "skolem"), (20, "skolem"), (21, "skolem"), (15, "langford"), (16, "langford"),
         (19, "langford"), (20, "langford"), (14, "hooked"), (15, "hooked")]


def _expected(n, variant):
    if variant == "hooked":
        return int(_load("oracle_counts.json")[f"hooked:{n}"]["ordered"])
    return int(_load("paper_counts.json")[variant][str(n)])


@pytest.mark.parametrize("lc,waves", [(27, 2048), (22, 6144), (22, 8192)])
def test_batched_persistent_launch_mixed_instances(lc, waves):
    """One persistent launch for Skolem 16, 17, 20, 21, Langford 15, 16, 19,
    20 and hooked 14, 15 (printed values, Tables 7 and 8; hooked from the
    oracle), in the untuned shape and in the shapes the autotuner picks for
    the benchmark (2^22 sign vectors per work item, 6144 or 8192 waves)."""
    counts, st = sk.count_batch(MIXED, tuning={"log2_chunk_terms": lc, "waves_per_launch": waves})
    assert st["launches"] == 1 and st["kernel_variant"] == 3
    for (n, v), c in zip(MIXED, counts):
        assert c == _expected(n, v), (v, n, c)


@pytest.mark.parametrize("lc,waves", [(24, 1024), (30, 4096)])
def test_batched_launch_shape_does_not_change_result(lc, waves):
    inst = [(16, "skolem"), (15, "langford"), (14, "hooked"), (17, "skolem")]
    counts, _ = sk.count_batch(inst, tuning={"log2_chunk_terms": lc, "waves_per_launch": waves})
    assert counts == [_expected(n, v) for n, v in inst]


def test_batch_with_unbatched_instances_and_zeros():
    inst = [(13, "skolem"), (12, "langford", sk.NO_SHORTCUT), (18, "skolem", sk.NO_SHORTCUT), (16, "skolem"),
            (14, "hooked", sk.ORDERED), (10, "skolem"), (15, "hooked", sk.VERIFY)]
    counts, st = sk.count_batch(inst)
    want = [1520280, 108144, 0, 700078384, _expected(14, "hooked"), 0, _expected(15, "hooked")]
    assert counts == want


def test_autotune_returns_a_working_shape():
    """The autotuner takes the sets count_batch takes: L(12) (no tuned body,
    a separate launch) and S(18) (no pairing, Sec. 1.1) are left out of the
    probes; a set with nothing to batch is an error."""
    inst = [(16, "skolem"), (16, "langford"), (15, "hooked"), (12, "langford"), (18, "skolem")]
    best, rate = sk.autotune_batch(inst)
    assert best["log2_chunk_terms"] >= 20 and best["waves_per_launch"] > 0 and rate > 0
    counts, _ = sk.count_batch(inst)
    assert counts == [_expected(n, v) for n, v in inst[:4]] + [0]
    with pytest.raises(sk.SkolemError) as e:
        sk.autotune_batch([(12, "langford"), (10, "skolem")])
    assert e.value.status == -7  # SK_ENOLIB


def test_l28_slice_chunks_match_cpu_recomputation():
    """Langford n = 28 at its full size (2^24 chunks of 2^31 sign vectors): the
    16 chunks of the 4096-chunk slice recomputed on the CPU by the oracle
    (tests/golden/l28_slice_chunks.json, written by make_l28_slice.py) must
    match bit for bit, in the launch the slice benchmark times."""
    with open(os.path.join(GOLD, "l28_slice_chunks.json")) as f:
        g = json.load(f)
    assert len(g["chunks"]) == 16
    ids = [c["id"] for c in g["chunks"]]
    assert set(ids) <= set(inputs.distinct_ids(g["slice_seed"], g["log2_chunks"], 4096))
    primes = g.get("primes", [g["prime"]])
    _say("l28 slice: 16 chunks of 2^31 terms, primes", len(primes))
    rows = sk.partial_chunks(g["n"], g["variant"], g["log2_chunks"], ids, primes)
    for c, row in zip(g["chunks"], rows):
        want = [int(c.get("residues", {}).get(str(p), c["residue"] if p == g["prime"] else -1)) for p in primes]
        assert row == want, c["id"]


@pytest.mark.parametrize("variant,n", [("skolem", 13), ("langford", 12), ("hooked", 11), ("skolem", 16),
                                       ("langford", 19), ("skolem", 17)])
def test_symmetry_reductions_equal_full_sum(variant, n):
    """The default count evaluates the half of the sign vectors with the top
    chunk variable (an even position) at +1 and doubles it (Lemma 2.4), and for
    Skolem and Langford weights the middle job variables by reversal (Lemma
    2.3); the full sum must give the same count."""
    _say("symmetry", variant, n)
    a = sk.count_ex(n, variant, ordered=True)
    b = sk.count_ex(n, variant, ordered=True, no_symmetry=True)
    assert a.count == b.count
    if n <= 13:
        assert a.count == O.count_backtrack(n, variant, threads=8)
    assert a.stats["symmetry_halved"] == 1 and b.stats["symmetry_halved"] == 0
    r = a.stats["reversal_quads"]
    if variant == "hooked" or a.stats["kernel_variant"] != 2:
        assert r == 0  # no reversal symmetry of the hooked position set; the reference body has no weights
    else:
        assert r == sk.describe(n, variant)["reversal_quads"] >= 1
    # evaluated: the Lemma 2.4 half, of which reversal keeps 1/2 + 2^-(r+1)
    assert a.stats["terms"] * 2 ** (r + 1) == b.stats["terms"] // 2 * (2 ** r + 1)


@pytest.mark.parametrize("variant,n,parts", [("skolem", 16, 8), ("langford", 15, 4), ("hooked", 14, 16),
                                             ("skolem", 12, 2), ("langford", 19, 32)])
def test_count_parts_combine_to_the_count(variant, n, parts):
    """A count split into independent parts (Sec. 2.2) and put together equals
    the count of one call; another split gives other rows, the same count."""
    _say("parts", variant, n, parts)
    rows = [sk.count_part(n, variant, k, parts, ordered=True)[0] for k in range(parts)]
    want = sk.count(n, variant, ordered=True)
    assert sk.count_combine(n, variant, rows, ordered=True) == want
    rows2 = [sk.count_part(n, variant, k, parts // 2, ordered=True)[0] for k in range(parts // 2)]
    assert sk.count_combine(n, variant, rows2, ordered=True) == want
    assert sk.count_combine(n, variant, rows) == (want if variant == "hooked" else want // 2)


def test_count_parts_reject_bad_splits():
    with pytest.raises(sk.SkolemError):
        sk.count_part(16, "skolem", 0, 3)   # not a power of two
    with pytest.raises(sk.SkolemError):
        sk.count_part(16, "skolem", 4, 4)   # part out of range
    with pytest.raises(sk.SkolemError):
        sk.count_part(16, "skolem", 0, 1 << 40)  # more parts than chunks


def test_caller_workspace_gives_the_same_results():
    """Counts and chunk rows with a caller-owned device workspace (a torch
    tensor sized by sk_workspace_bytes / sk_partial_workspace_bytes) equal
    those with the library's own; a workspace one byte short is refused with
    SK_ENOMEM before any work and leaves the outputs untouched."""
    import ctypes
    import torch
    inst = [(16, "skolem"), (15, "langford"), (14, "hooked", sk.ORDERED), (13, "skolem")]
    nb = sk.workspace_bytes(inst)
    ws = torch.empty(nb, dtype=torch.uint8, device="cuda")
    want = [_expected(16, "skolem"), _expected(15, "langford"), _expected(14, "hooked"), 1520280]
    got, _ = sk.count_batch(inst, workspace=ws)
    assert got == want
    assert sk.count_ex(13, "skolem", workspace=ws).count == 1520280
    ids = inputs.distinct_ids(77, 10, 300)
    rows = sk.partial_chunks(16, "skolem", 10, ids, PRIMES[:2])
    pb = sk.partial_workspace_bytes(16, "skolem", len(ids), 2)
    wp = torch.empty(pb, dtype=torch.uint8, device="cuda")
    assert sk.partial_chunks(16, "skolem", 10, ids, PRIMES[:2], workspace=wp) == rows
    # too small: SK_ENOMEM, outputs untouched
    L = sk.lib()
    arr = sk._instances(inst)
    out = (sk.U128 * len(inst))()
    for o in out:
        o.lo, o.hi = 7, 7
    st = L.sk_count_batch(arr, len(inst), None, ctypes.c_void_p(ws.data_ptr()), nb - 1, None, None, out)
    assert st == -5 and all(o.lo == 7 and o.hi == 7 for o in out)
    with pytest.raises(sk.SkolemError) as ei:
        sk.partial_chunks(16, "skolem", 10, ids, PRIMES[:2], workspace=(wp.data_ptr(), pb - 1))
    assert ei.value.status == -5
    torch.cuda.synchronize()


def test_batch_groups_and_one_prime_per_item():
    """Instances of three batched groups in one call (n = 12, 13; the other
    14 <= n <= 21; the mixed set), one persistent launch per group: printed
    and stored oracle values, sums that must vanish where no pairing exists
    (shortcut off), and hooked n = 18 against its separate count.  Then the
    mixed set with one prime per work item (group 1's second kernel)."""
    g = _load("oracle_counts.json")
    h18 = sk.count(18, "hooked", ordered=True)
    inst = [(12, "skolem"), (13, "skolem"), (12, "langford"), (13, "hooked", sk.ORDERED),
            (18, "skolem", sk.NO_SHORTCUT), (17, "langford", sk.NO_SHORTCUT), (16, "hooked", sk.NO_SHORTCUT),
            (18, "hooked", sk.ORDERED), (16, "skolem"), (15, "langford")]
    counts, st = sk.count_batch(inst, tuning={"log2_chunk_terms": 24, "waves_per_launch": 4096})
    want = [227968, 1520280, 108144, int(g["hooked:13"]["ordered"]), 0, 0, 0, h18, 700078384, 39809640]
    assert counts == want
    # three group launches, and one reference-body launch for L(12), whose walk
    # is too short for the tuned body
    assert sk.describe(12, "langford")["n_walk"] < 5
    assert st["launches"] == 4
    one, st1 = sk.count_batch(MIXED, tuning={"log2_chunk_terms": 24, "waves_per_launch": 4096, "primes_per_item": 1})
    assert one == [_expected(n, v) for n, v in MIXED]
    assert st1["launches"] == 1
