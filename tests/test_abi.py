"""The C ABI library loads and exports every entry point include/skolem.h
declares; host-only helpers work without a GPU."""
import ctypes
import os
import re

import pytest

import paper_1507_00315_amd as sk

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    text = open(os.path.join(ROOT, "include", "skolem.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(sk_[a-z0-9_]+)\s*\(", text)))


def test_library_present_and_exports_every_declared_symbol():
    L = sk.lib()
    names = _declared()
    assert "sk_count" in names and "sk_partial_chunks" in names
    for name in names:
        assert hasattr(L, name), name
    assert set(names) <= set(sk.EXPORTED), sorted(set(names) - set(sk.EXPORTED))


def test_strerror_and_decimal_are_host_only():
    L = sk.lib()
    assert L.sk_strerror(0) == b"ok"
    assert L.sk_strerror(-4) == b"self-check failed"
    buf = ctypes.create_string_buffer(64)
    x = sk.U128(0xFFFFFFFFFFFFFFFF, 0x1)
    n = L.sk_u128_to_decimal(x, buf, 64)
    assert buf.value.decode() == str((1 << 65) - 1) and n == len(buf.value)
    assert L.sk_u128_to_decimal(x, buf, 5) == -1


def test_chunk_bits_planning_is_host_only():
    # host planner: x_1 fixed, six lane variables, walked variables share no
    # pair with the lane variables, the rest are job variables.
    for n, v in [(12, 0), (24, 0), (28, 1), (15, 2)]:
        c = sk.max_chunk_bits(n, v)
        assert 0 <= c <= 2 * n - 7
    assert sk.max_chunk_bits(0, 0) < 0 and sk.max_chunk_bits(40, 0) < 0


def test_no_gpu_reports_device_error_not_fallback():
    try:
        import torch
        has_gpu = torch.cuda.is_available()
    except Exception:
        has_gpu = False
    if has_gpu:
        pytest.skip("GPU present")
    with pytest.raises(sk.SkolemError) as ei:
        sk.count(8, "skolem")
    assert ei.value.status in (-3,)


def test_network_size_and_init_are_host_only():
    # 130 -> 256 -> 256 -> 32 x 64 for Skolem n = 32
    assert sk.mlp_param_count(32, "skolem") == 130 * 256 + 256 + 256 * 256 + 256 + 2048 * 256 + 2048 == 625664
    assert sk.mlp_param_count(31, "hooked", 16, 8) == (63 + 62 + 2) * 16 + 16 + 16 * 8 + 8 + 31 * 63 * 8 + 31 * 63
    assert sk.mlp_param_count(33, "skolem") == 0
    a = sk.mlp_init(32, "skolem", seed=4)
    b = sk.mlp_init(32, "skolem", seed=4)
    assert (a == b).all() and not (a == sk.mlp_init(32, "skolem", seed=5)).all()
    W1 = a[:256 * 130]
    assert abs(W1.std() * (130 ** 0.5) - 1.0) < 0.02 and abs(W1.mean()) < 0.01
    assert (a[256 * 130:256 * 131] == 0).all()  # b1


def test_lemma_2_4_symmetry_matches_existence_conditions():
    # negating the even positions leaves the term invariant exactly when the
    # existence conditions of Sec. 1.1 hold (host-side plan, no GPU)
    for n in range(2, 33):
        for v, ok in (("skolem", n % 4 in (0, 1)), ("langford", n % 4 in (0, 3)), ("hooked", n % 4 in (2, 3))):
            if v == "hooked" and n > 31:
                continue
            assert sk.describe(n, v)["symmetric"] == int(ok), (v, n)


def test_prime_count_covers_the_count_bound():
    # the library's k primes (the largest below 2^46) must exceed n! * 2^8, and
    # k - 1 of them must not (fewest primes); checked with exact integers
    import math
    import oracle as O
    O.build(force=False)
    primes = O.primes_below(1 << 46, 4)
    for v in ("skolem", "langford"):
        for n in range(1, 33):
            k = sk.describe(n, v)["primes"]
            bound = math.factorial(n) << 8
            assert math.prod(primes[:k]) > bound, (v, n, k)
            assert k == 1 or math.prod(primes[:k - 1]) <= bound, (v, n, k)


def test_reversal_quadruples_for_skolem_and_langford_only():
    # Lemma 2.3 needs a position set symmetric under i -> 2n + 1 - i
    for n in range(12, 33):
        for v in ("skolem", "langford"):
            r = sk.describe(n, v)["reversal_quads"]
            assert r >= 2 and (r == 4 or n < 15), (v, n, r)  # from n = 15 on the walk is n - 9 variables
        if n <= 31:
            assert sk.describe(n, "hooked")["reversal_quads"] == 0


def test_count_combine_is_host_only():
    import oracle as O
    O.build(force=False)
    primes = O.primes_below(1 << 46, 4)
    # no pairing exists: the count is 0 whatever the parts hold
    assert sk.count_combine(10, "skolem", [[0, 0]] * 4) == 0
    # a residue out of range is rejected
    k = sk.describe(12, "skolem")["primes"]
    with pytest.raises(sk.SkolemError):
        sk.count_combine(12, "skolem", [[primes[i] for i in range(k)]])
    # the ordered count C enters as C * 2^(2n - 1 - halved) modulo each prime
    n = 12
    d = sk.describe(n, "skolem")
    C = 455936
    rows = [[C * pow(2, 2 * n - 1 - d["halved"], primes[i]) % primes[i] for i in range(k)]]
    assert sk.count_combine(n, "skolem", rows) == C // 2
    assert sk.count_combine(n, "skolem", rows, ordered=True) == C
    # split into parts: any additive split of the residues gives the same count
    split = [[(r * 3) % primes[i] for i, r in enumerate(rows[0])],
             [(r * -2) % primes[i] for i, r in enumerate(rows[0])]]
    assert sk.count_combine(n, "skolem", split, ordered=True) == C


def test_bench_refuses_more_than_one_gpu():
    import subprocess
    import sys
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2 and "one GPU only" in r.stderr and r.stdout == ""


def test_workspace_sizes_are_host_only():
    # counts: the 128-bit accumulators of one batched launch and its counter,
    # the same for every instance set; 0 on a bad instance
    a = sk.workspace_bytes([(20, "skolem")])
    b = sk.workspace_bytes([(16, "skolem"), (15, "langford"), (14, "hooked", sk.ORDERED)])
    assert a == b and 16 * 4 * 16 <= a <= 4096
    assert sk.workspace_bytes([(40, "skolem")]) == 0
    # listed chunks: accumulators and the work-queue counter (256 + 256), then
    # per chunk of a launch one row of up to four 128-bit sums and one chunk
    # id, each region rounded to 256 bytes
    t = {"waves_per_launch": 64}
    assert sk.partial_workspace_bytes(20, "skolem", 1000, 2, t) == 512 + 64 * 64 + 512
    assert sk.partial_workspace_bytes(20, "skolem", 10, 2, t) == 512 + 768 + 256
    assert sk.partial_workspace_bytes(20, "skolem", 10, 9, t) == 0


def _rows(n, variant, C):
    """Residue row of the ordered count C as the GPU sum delivers it:
    C * 2^(2n - 1 - halved) modulo each of the count's primes."""
    import oracle as O
    O.build(force=False)
    d = sk.describe(n, variant)
    primes = O.primes_below(1 << 46, d["primes"])
    return [C * pow(2, 2 * n - 1 - d["halved"], p) % p for p in primes], primes


@pytest.mark.parametrize("variant,n,ordered", [("skolem", 12, 455936), ("skolem", 24, 204776117691241344),
                                               ("langford", 23, 7598911885030976)])
def test_corrupted_residue_is_rejected(variant, n, ordered):
    """A residue set changed in any one prime gives a CRT value that is
    uniform-looking in [0, prod p); it passes the bound check C <= n! (and the
    parity check of the reflections) with probability about n! / prod p:
    2^-63 for n = 12, 2^-12 for n = 24 with two primes.  Seeded corruptions
    of one residue (plus 1, minus 1, random) must all give SK_ECHECK."""
    from paper_1507_00315_amd import inputs
    row, primes = _rows(n, variant, ordered)
    assert sk.count_combine(n, variant, [row], ordered=True) == ordered
    rng = inputs.SplitMix64(4000 + n)
    bad = []
    for i, p in enumerate(primes):
        for delta in (1, p - 1, 1 + rng.below(p - 1), 1 + rng.below(p - 1)):
            r = list(row)
            r[i] = (r[i] + delta) % p
            bad.append(r)
    for r in bad:
        with pytest.raises(sk.SkolemError) as ei:
            sk.count_combine(n, variant, [r])
        assert ei.value.status == -4  # SK_ECHECK
