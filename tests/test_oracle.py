"""Pins for the CPU oracle against what the paper and the mathematics fix.

Every check here runs on the CPU.  Sources:
* Sec. 2.1 worked example (the six sequences of order 4, coefficient 6),
* Sec. 1.1 example pairings, Tables 1 and 2 (constructions),
* Table 7 and Table 8 exact values (small n),
* existence conditions (Sec. 1.1),
* brute force and Algorithm 1 / Lemma 2.1 on tiny instances,
* Lemmas 2.2 and 2.4 as identities between partial sums.
"""
import json
import os
import random

import pytest

import oracle as O

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _load(name):
    with open(os.path.join(GOLD, name)) as f:
        return json.load(f)


@pytest.fixture(scope="module", autouse=True)
def _built():
    O.build(force=False)


# ---------------------------------------------------------------- Sec. 2.1

def test_worked_example_n4_lists_exactly_the_six_sequences():
    g = _load("worked_example_n4.json")
    got = sorted(O.labels(p, 4, "skolem") for p in O.enumerate_pairings(4, "skolem"))
    assert got == sorted(g["sequences"])
    assert O.count_backtrack(4, "skolem") == g["coefficient"]
    assert O.algorithm1(4, "skolem") == g["coefficient"]


def test_section_1_1_examples_are_valid():
    g = _load("worked_example_n4.json")
    assert O.is_valid_pairing([tuple(x) for x in g["skolem_n4_pairs"]], 4, "skolem")
    pairs5 = O.sequence_to_pairs(g["skolem_n5_sequence"], 5)
    assert O.is_valid_pairing(pairs5, 5, "skolem")
    assert sorted(pairs5) == sorted(tuple(x) for x in g["skolem_n5_pairs"])
    lp = O.sequence_to_pairs(g["langford_n4_sequence"], 4)
    assert O.is_valid_pairing(lp, 4, "langford")
    # the Skolem reading of the Langford example is not valid (spacing differs)
    assert not O.is_valid_pairing(lp, 4, "skolem")


def test_checker_rejects_corruptions():
    good = O.skolem_construction(8)
    assert O.is_valid_pairing(good, 8, "skolem")
    bad = list(good)
    a, b = bad[2]
    bad[2] = (a + 1, b + 1)
    assert not O.is_valid_pairing(bad, 8, "skolem")
    bad = list(good)
    bad[0], bad[1] = bad[1], bad[0]
    assert not O.is_valid_pairing(bad, 8, "skolem")


# ------------------------------------------------------- Tables 7 and 8

@pytest.mark.parametrize("n", [4, 5, 8, 9, 12, 13])
def test_printed_skolem_values_small(n):
    g = _load("paper_counts.json")["skolem"]
    assert O.reported(O.count_backtrack(n, "skolem", threads=8), n, "skolem") == int(g[str(n)])


@pytest.mark.parametrize("n", [3, 4, 7, 8, 11, 12])
def test_printed_langford_values_small(n):
    g = _load("paper_counts.json")["langford"]
    assert O.reported(O.count_backtrack(n, "langford", threads=8), n, "langford") == int(g[str(n)])


def test_n1_conventions():
    """n = 1 (Sec. 1.3 halves for reflections only when n > 1): the single
    Skolem pairing (1, 2) is its own reflection, so S(1) = 1 = C(1); no
    Langford pairing has positions 1, 2 at distance 2, so L(1) = 0; the hooked
    set {1, 3} holds the pair (1, 3) only at distance 2, so H(1) = 0."""
    assert O.enumerate_pairings(1, "skolem") == [(1,)]
    assert O.count_backtrack(1, "skolem") == 1 and O.reported(1, 1, "skolem") == 1
    assert O.count_backtrack(1, "langford") == 0 and O.reported(0, 1, "langford") == 0
    assert O.count_backtrack(1, "hooked") == 0
    # n > 1: every pairing has a distinct reflection, so ordered counts are even
    assert O.reported(6, 4, "skolem") == 3 and O.reported(2, 3, "langford") == 1
    with pytest.raises(AssertionError):
        O.reported(7, 4, "skolem")


def test_table4_ordered_is_twice_reported():
    g = _load("paper_counts.json")
    for n, v in g["skolem_ordered"].items():
        if not n.startswith("_"):
            assert int(v) == 2 * int(g["skolem"][n])
    for n, v in g["langford_ordered"].items():
        if not n.startswith("_"):
            assert int(v) == 2 * int(g["langford"][n])


# ------------------------------------------------------------ existence

@pytest.mark.parametrize("variant", ["skolem", "langford", "hooked"])
def test_existence_zeros(variant):
    for n in range(1, 12):
        c = O.count_backtrack(n, variant, threads=4)
        assert (c > 0) == O.exists(n, variant), (variant, n, c)


# --------------------------------------------------------- constructions

def test_skolem_construction_table1_valid_and_found():
    for n in range(8, 30):
        if n % 4 in (0, 1):
            assert O.is_valid_pairing(O.skolem_construction(n), n, "skolem"), n
    for n in (8, 9):
        left_ends = tuple(a for a, _ in O.skolem_construction(n))
        assert left_ends in set(O.enumerate_pairings(n, "skolem"))


def test_davies_construction_table2_valid_and_found():
    for n in range(3, 29):
        if n % 4 in (0, 3):
            pr = O.sequence_to_pairs(O.davies_construction(n), n)
            assert pr is not None and O.is_valid_pairing(pr, n, "langford"), n
    assert O.davies_construction(4) == _load("worked_example_n4.json")["langford_n4_sequence"]
    for n in (7, 8):
        left_ends = tuple(a for a, _ in O.sequence_to_pairs(O.davies_construction(n), n))
        assert left_ends in set(O.enumerate_pairings(n, "langford"))


# ------------------------------------------ brute force, Algorithm 1

@pytest.mark.parametrize("variant", ["skolem", "langford", "hooked"])
def test_backtrack_equals_bruteforce_and_enumeration(variant):
    for n in range(1, 7):
        c = O.count_backtrack(n, variant)
        assert c == O.count_bruteforce(n, variant), (variant, n)
        assert c == len(O.enumerate_pairings(n, variant))


@pytest.mark.parametrize("variant", ["skolem", "langford", "hooked"])
def test_algorithm1_equals_backtrack(variant):
    for n in range(1, 8):
        assert O.algorithm1(n, variant) == O.count_backtrack(n, variant), (variant, n)


def test_hooked_small_values():
    # hand check: H(2) = 1, pairs (3,5) and (1,2); H(1) = 0.
    assert O.enumerate_pairings(2, "hooked") == [(1, 3)]
    assert O.count_backtrack(1, "hooked") == 0


# ------------------------------------------- partial sums (Lemma 2.1)

P3 = O.primes_below(1 << 46, 3)


def _random_fixed(n, variant, nfix, rng, include_first=True):
    pos, _ = O.instance(n, variant)
    pick = rng.sample(pos[1:], nfix - 1) if include_first else rng.sample(pos, nfix)
    fixed = {q: rng.choice((1, -1)) for q in pick}
    if include_first:
        fixed[pos[0]] = 1
    return fixed


@pytest.mark.parametrize("variant", ["skolem", "langford", "hooked"])
def test_gray_partial_equals_direct_partial(variant):
    rng = random.Random(1507)
    for n in (5, 6, 7, 8):
        for _ in range(3):
            fixed = _random_fixed(n, variant, rng.randint(1, 5), rng)
            for p in P3[:2] + [1000003]:
                a = O.chunk_partial(n, variant, fixed, p, "direct")
                b = O.chunk_partial(n, variant, fixed, p, "gray", threads=3)
                assert a == b, (variant, n, fixed, p)


@pytest.mark.parametrize("variant", ["skolem", "langford", "hooked"])
def test_full_sum_is_count_times_power_of_two(variant):
    """Lemma 2.1 with x_1 fixed (Lemma 2.2): sum = C * 2^(m-1)."""
    for n in range(1, 12):
        pos, _ = O.instance(n, variant)
        m = len(pos)
        c = O.count_backtrack(n, variant, threads=4)
        for p in P3:
            h = O.chunk_partial(n, variant, {1: 1}, p, "gray", threads=8)
            assert h == c * pow(2, m - 1, p) % p, (variant, n, p)


@pytest.mark.parametrize("variant", ["skolem", "langford", "hooked"])
def test_negation_symmetry_lemma_2_2(variant):
    rng = random.Random(7)
    for n in (6, 7, 8, 9):
        fixed = _random_fixed(n, variant, 4, rng, include_first=False)
        neg = {q: -v for q, v in fixed.items()}
        p = P3[0]
        assert (O.chunk_partial(n, variant, fixed, p, "gray", 2) ==
                O.chunk_partial(n, variant, neg, p, "gray", 2))


@pytest.mark.parametrize("variant", ["skolem", "langford", "hooked"])
def test_even_position_symmetry_lemma_2_4(variant):
    """Negating every even position multiplies each term by
    (-1)^(#even positions + #odd differences); +1 exactly when pairings can
    exist, so chunk partials pair up (and the total vanishes otherwise)."""
    rng = random.Random(11)
    for n in range(3, 10):
        pos, d = O.instance(n, variant)
        eps = (-1) ** (sum(1 for q in pos if q % 2 == 0) + sum(1 for x in d if x % 2 == 1))
        assert (eps == 1) == O.exists(n, variant)
        fixed = _random_fixed(n, variant, 5, rng)
        hat = {q: (-v if q % 2 == 0 else v) for q, v in fixed.items()}
        p = P3[1]
        a = O.chunk_partial(n, variant, fixed, p, "gray", 2)
        b = O.chunk_partial(n, variant, hat, p, "gray", 2)
        assert b == (a if eps == 1 else (-a) % p), (variant, n)


@pytest.mark.parametrize("variant", ["skolem", "langford"])
def test_reversal_symmetry_lemma_2_3(variant):
    """Reversal x_i -> x_(2n+1-i) leaves prod x and F unchanged (Lemma 2.3);
    followed by a global negation when x_2n = -1 (Lemma 2.2) it keeps x_1 =
    +1.  So the partial sum with x_1 = +1, x_2n = s and x_q = s_q fixed equals
    the one with x_2n = s and x_(2n+1-q) = s * s_q fixed -- the identity the
    reversal weights of the exact count rely on."""
    rng = random.Random(23)
    p = P3[2]
    for n in range(4, 10):
        pos, _ = O.instance(n, variant)
        top = 2 * n
        for _ in range(3):
            s_top = rng.choice((1, -1))
            inner = rng.sample(range(2, top), 4)
            fixed = {1: 1, top: s_top}
            fixed.update({q: rng.choice((1, -1)) for q in inner})
            image = {1: 1, top: s_top}
            image.update({top + 1 - q: s_top * v for q, v in fixed.items() if q not in (1, top)})
            a = O.chunk_partial(n, variant, fixed, p, "gray", 2)
            b = O.chunk_partial(n, variant, image, p, "gray", 2)
            assert a == b, (variant, n, fixed, image)


def test_primes():
    assert O.is_prime(2 ** 61 - 1) and O.is_prime(2 ** 31 - 1)
    assert not O.is_prime(2 ** 61 + 1) and not O.is_prime(561) and not O.is_prime(3215031751)
    ps = O.primes_below(1 << 20, 5)
    assert all(O.is_prime(x) for x in ps) and len(set(ps)) == 5
    assert all(not O.is_prime(x) for x in range(ps[0] + 1, 1 << 20))


# ---------------------------------------------------------------- Sec. 2, inclusion-exclusion

def test_larsen_hand_computed_small_cases():
    """n = 1: only S = {} contributes (one placement).  n = 2 Skolem on
    positions 1..4, d = 1, 2: S = {} gives 3 * 2 = 6; S = {1}, {2}, {3}, {4}
    give 2*1, 1*1, 1*1, 2*1; no two positions host both pairs: 6 - 6 = 0.
    n = 4 Skolem: the worked example's 6 ordered pairings (Sec. 2.1)."""
    assert O.larsen_literal(1, "skolem") == 1
    assert O.larsen_literal(2, "skolem") == 0
    assert O.larsen_literal(4, "skolem") == 6
    assert O.larsen_literal(3, "langford") == 2


@pytest.mark.parametrize("variant", ["skolem", "langford", "hooked"])
def test_larsen_literal_equals_backtrack(variant):
    for n in range(1, 8):
        assert O.larsen_literal(n, variant) == O.count_backtrack(n, variant), (variant, n)


@pytest.mark.parametrize("variant", ["skolem", "langford", "hooked"])
def test_larsen_modular_equals_backtrack(variant):
    p = O.primes_below(1 << 46, 1)[0]
    for n in range(1, 12):
        assert O.larsen_count(n, variant, p, threads=8) == O.count_backtrack(n, variant, threads=8), (variant, n)
        if n <= 7:
            assert O.larsen_count(n, variant, p) == O.larsen_literal(n, variant) % p


def test_larsen_printed_s12_and_partials_add_up():
    """S(12) = 227968 (Table 7), ordered 455936; splitting on any position
    (occupied or forced empty) splits the sum."""
    p = O.primes_below(1 << 46, 1)[0]
    assert O.larsen_count(12, "skolem", p, threads=8) == 2 * 227968
    for q in (1, 7, 18):
        a = O.larsen_partial(9, "langford", {q: 0}, p)
        b = O.larsen_partial(9, "langford", {q: 1}, p)
        assert (a + b) % p == O.count_backtrack(9, "langford") % p
    # a restriction of the C sum equals the same restriction of the literal
    # Python sum (position 1 forced empty)
    pos, d = O.instance(5, "skolem")
    want = 0
    for bits in range(1 << 9):
        S = {pos[1 + i] for i in range(9) if (bits >> i) & 1} | {pos[0]}
        T = [a for a in pos if a not in S]
        prod = 1
        for dk in d:
            prod *= sum(1 for a in T if a + dk in T)
        want += -prod if len(S) % 2 else prod
    assert O.larsen_partial(5, "skolem", {1: 0}, p) == want % p
