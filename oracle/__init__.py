"""CPU oracle for the exact counts and the tempering estimator.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import this package.  It shares no code
with the GPU library in ``paper_1507_00315_amd`` and imports nothing from it.

What is here, and the passage of arXiv 1507.00315 each part follows:

* ``instance``            -- the problems: Skolem pairings (Sec. 1.1: split 1..2n
  into pairs with differences 1..n), Langford pairings (Sec. 1.1: the two copies
  of k have k numbers between them, so positions differ by k+1) and hooked Skolem
  pairings (Sec. 1.2: positions 1..2n-1 and 2n+1).
* ``count_backtrack``     -- the plain definition of the ordered count, by the
  backtracking search of Sec. 2 (largest difference placed first), in C.
* ``count_bruteforce``    -- every placement of every pair tried (tiny n).
* ``enumerate_pairings``  -- the pairings themselves (tiny n), for the worked
  example of Sec. 2.1.
* ``algorithm1``          -- Algorithm 1 / Lemma 2.1 taken literally: the signed
  sum over all of {+1,-1}^P with exact Python integers, divided by 2^|P|.
* ``chunk_partial``       -- the signed sum of Lemma 2.1 over the sign vectors that
  agree with a fixed partial assignment, modulo p (C; plain or Gray-code order).
* ``larsen_literal``, ``larsen_partial``, ``larsen_count`` -- the inclusion-
  exclusion count of Sec. 2 (third approach: placements avoiding positions),
  literally with exact integers (tiny n) and modulo p in C, each term from
  scratch.
* ``skolem_construction`` / ``davies_construction`` -- Tables 1 and 2.
* ``reported``            -- the counting conventions of Sec. 1.3 (reflections
  counted once for n > 1).

Parity unpinned: nothing in this file.  Every function is pinned by a test in
``tests/test_oracle.py`` against values or properties the paper or the
mathematics fix.
"""
from __future__ import annotations

import ctypes
import itertools
import math
import os
import subprocess
from typing import Dict, List, Optional, Sequence, Tuple

HERE = os.path.dirname(os.path.abspath(__file__))
_SRCS = [os.path.join(HERE, "skolem_oracle.c"), os.path.join(HERE, "pt_oracle.c")]
_LIB = os.path.join(HERE, "liboracle.so")

SKOLEM, LANGFORD, HOOKED = 0, 1, 2
VARIANTS = {"skolem": SKOLEM, "langford": LANGFORD, "hooked": HOOKED}


def _variant(v) -> int:
    if isinstance(v, str):
        return VARIANTS[v.lower()]
    return int(v)


# --------------------------------------------------------------------------
# Build and load the C part
# --------------------------------------------------------------------------

def _stale() -> bool:
    if not os.path.exists(_LIB):
        return True
    t = os.path.getmtime(_LIB)
    return any(os.path.getmtime(s) > t for s in _SRCS)


def build(force: bool = True) -> str:
    """Compile the C sources into ``liboracle.so`` with gcc."""
    if force or _stale():
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-pthread",
                               "-o", tmp] + _SRCS + ["-lm"])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        if _stale():
            build(force=True)
        L = ctypes.CDLL(_LIB)
        L.orc_count_backtrack.restype = ctypes.c_uint64
        L.orc_count_backtrack.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int]
        L.orc_chunk_partial_direct.restype = ctypes.c_uint64
        L.orc_chunk_partial_direct.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_uint64,
                                               ctypes.c_uint64, ctypes.c_uint64]
        L.orc_chunk_partial_gray.restype = ctypes.c_uint64
        L.orc_chunk_partial_gray.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_uint64,
                                             ctypes.c_uint64, ctypes.c_uint64, ctypes.c_int]
        u32p = ctypes.POINTER(ctypes.c_uint32)
        u64p = ctypes.POINTER(ctypes.c_uint64)
        ip = ctypes.POINTER(ctypes.c_int)
        L.orc_larsen_partial.restype = ctypes.c_uint64
        L.orc_larsen_partial.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_uint64, ctypes.c_uint64,
                                         ctypes.c_uint64, ctypes.c_int]
        L.orc_philox4x32_10.argtypes = [u32p, u32p, u32p]
        L.orc_philox4x32_10.restype = None
        L.orc_energy_histogram.argtypes = [ctypes.c_int, ctypes.c_int, u64p]
        L.orc_energy_histogram.restype = ctypes.c_int
        L.orc_pt_ladder.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.POINTER(ctypes.c_double),
                                    ctypes.c_uint64, ctypes.c_uint64, ctypes.c_uint32, ctypes.c_int,
                                    u64p, u64p, u64p, u64p, ip, ip]
        L.orc_pt_ladder.restype = ctypes.c_int
        _lib = L
    return _lib


# --------------------------------------------------------------------------
# Problem statement
# --------------------------------------------------------------------------

def instance(n: int, variant) -> Tuple[List[int], List[int]]:
    """(positions, differences) for the variant, positions 1-based ascending."""
    v = _variant(variant)
    if n < 1:
        raise ValueError("n must be >= 1")
    if v == HOOKED:
        pos = list(range(1, 2 * n)) + [2 * n + 1]
    else:
        pos = list(range(1, 2 * n + 1))
    diffs = [k + 1 if v == LANGFORD else k for k in range(1, n + 1)]
    return pos, diffs


def reported(ordered: int, n: int, variant) -> int:
    """Convention of Sec. 1.3: reflections counted once (Skolem and Langford,
    n > 1; no pairing is its own reflection).  A hooked pairing's reflection is
    not a hooked pairing, so hooked counts are not halved."""
    v = _variant(variant)
    if v == HOOKED:
        return ordered
    if v == SKOLEM and n == 1:
        return ordered
    assert ordered % 2 == 0
    return ordered // 2


def exists(n: int, variant) -> bool:
    """Existence conditions: Skolem iff n = 0,1 mod 4; Langford iff n = 0,3
    mod 4 (Sec. 1.1); hooked iff n = 2,3 mod 4 (position-sum parity)."""
    v = _variant(variant)
    r = n % 4
    return r in ((0, 1) if v == SKOLEM else (0, 3) if v == LANGFORD else (2, 3))


# --------------------------------------------------------------------------
# Counting by search
# --------------------------------------------------------------------------

def count_backtrack(n: int, variant, threads: int = 1) -> int:
    """Ordered count (reflections distinct), backtracking in C."""
    return int(lib().orc_count_backtrack(n, _variant(variant), threads))


def enumerate_pairings(n: int, variant) -> List[Tuple[int, ...]]:
    """Every ordered pairing as the tuple (a_1, ..., a_n) of left ends."""
    pos, d = instance(n, variant)
    free = set(pos)
    out: List[Tuple[int, ...]] = []
    a = [0] * n

    def rec(k: int) -> None:
        if k < 0:
            out.append(tuple(a))
            return
        for s in sorted(free):
            if s + d[k] in free:
                free.discard(s)
                free.discard(s + d[k])
                a[k] = s
                rec(k - 1)
                free.add(s)
                free.add(s + d[k])

    rec(n - 1)
    return out


def count_bruteforce(n: int, variant) -> int:
    """Tries every combination of left ends; counts those that cover P."""
    pos, d = instance(n, variant)
    pset = set(pos)
    choices = [[a for a in pos if a + dk in pset] for dk in d]
    total = 0
    for combo in itertools.product(*choices):
        used = set()
        ok = True
        for a, dk in zip(combo, d):
            if a in used or a + dk in used:
                ok = False
                break
            used.add(a)
            used.add(a + dk)
        if ok and used == pset:
            total += 1
    return total


def labels(pairing: Sequence[int], n: int, variant) -> List[int]:
    """Sequence notation: entry at each position is the label k of its pair."""
    pos, d = instance(n, variant)
    seq: Dict[int, int] = {}
    for k, (a, dk) in enumerate(zip(pairing, d), start=1):
        seq[a] = k
        seq[a + dk] = k
    return [seq[p] for p in pos]


def is_valid_pairing(pairs: Sequence[Tuple[int, int]], n: int, variant) -> bool:
    """pairs[k-1] = (a, b) for label k: checks b - a = d_k and that the 2n
    numbers are exactly the position set."""
    pos, d = instance(n, variant)
    if len(pairs) != n:
        return False
    used: List[int] = []
    for (a, b), dk in zip(pairs, d):
        if b - a != dk:
            return False
        used += [a, b]
    return sorted(used) == sorted(pos)


# --------------------------------------------------------------------------
# Algorithm 1 / Lemma 2.1, literally
# --------------------------------------------------------------------------

def algorithm1(n: int, variant) -> int:
    """Sum over all x in {+1,-1}^P of (prod x) * prod_k sum_{i} x_i x_{i+d_k},
    with exact integers, divided by 2^|P| (Lemma 2.1).  Returns the ordered
    count.  Exponential: use |P| <= 16."""
    pos, d = instance(n, variant)
    m = len(pos)
    idx = {p: i for i, p in enumerate(pos)}
    total = 0
    for bits in range(1 << m):
        x = [(-1 if (bits >> i) & 1 else 1) for i in range(m)]
        sign = 1
        for v in x:
            sign *= v
        prod = 1
        for dk in d:
            s = 0
            for p in pos:
                q = p + dk
                if q in idx:
                    s += x[idx[p]] * x[idx[q]]
            prod *= s
        total += sign * prod
    assert total % (1 << m) == 0
    return total // (1 << m)


# --------------------------------------------------------------------------
# Partial sign-vector sums modulo p
# --------------------------------------------------------------------------

def chunk_partial(n: int, variant, fixed: Dict[int, int], p: int, method: str = "gray",
                  threads: int = 1) -> int:
    """Residue in [0, p) of the signed sum over the sign vectors that take the
    values ``fixed`` ({position: +1 or -1}) at the fixed positions."""
    mask = 0
    neg = 0
    for q, val in fixed.items():
        if val not in (1, -1):
            raise ValueError("fixed values are +1 or -1")
        mask |= 1 << (q - 1)
        if val == -1:
            neg |= 1 << (q - 1)
    v = _variant(variant)
    if method == "direct":
        return int(lib().orc_chunk_partial_direct(n, v, mask, neg, p))
    if method == "gray":
        return int(lib().orc_chunk_partial_gray(n, v, mask, neg, p, threads))
    raise ValueError(method)


# --------------------------------------------------------------------------
# Inclusion-exclusion (Sec. 2, the third approach)
# --------------------------------------------------------------------------

def larsen_literal(n: int, variant) -> int:
    """Ordered count by inclusion-exclusion over the positions left empty,
    with exact integers: the universe is every placement of the pairs inside
    P with overlaps allowed, A_i those leaving position i empty, and the
    pairings are the placements in no A_i, so
    C = sum over S subset of P of (-1)^|S| prod_k N_k(P minus S), N_k(T) being
    the number of a with a, a + d_k in T.  Exponential: use |P| <= 16."""
    pos, d = instance(n, variant)
    m = len(pos)
    total = 0
    for bits in range(1 << m):
        T = {pos[i] for i in range(m) if not (bits >> i) & 1}
        prod = 1
        for dk in d:
            prod *= sum(1 for a in T if a + dk in T)
            if prod == 0:
                break
        total += -prod if bin(bits).count("1") % 2 else prod
    return total


def larsen_partial(n: int, variant, fixed: Dict[int, int], p: int, threads: int = 1) -> int:
    """Residue in [0, p) of the inclusion-exclusion sum restricted to the sets
    S that agree with ``fixed`` ({position: 1 if the position is occupied
    (not in S), 0 if it is in S}), each term evaluated from scratch (C)."""
    mask = 0
    empty = 0
    for q, val in fixed.items():
        if val not in (0, 1):
            raise ValueError("fixed values are 0 (in S) or 1 (not in S)")
        mask |= 1 << (q - 1)
        if val == 0:
            empty |= 1 << (q - 1)
    return int(lib().orc_larsen_partial(n, _variant(variant), mask, empty, p, threads))


def larsen_count(n: int, variant, p: int, threads: int = 1) -> int:
    """The whole inclusion-exclusion sum modulo p (the ordered count when
    p exceeds it)."""
    return larsen_partial(n, variant, {}, p, threads)


# --------------------------------------------------------------------------
# Constructions (Tables 1 and 2)
# --------------------------------------------------------------------------

def skolem_construction(n: int) -> List[Tuple[int, int]]:
    """Table 1 (Skolem's construction) for n = 4k and n = 4k + 1, k >= 2.
    Returns pairs (a, b) listed by label k = b - a."""
    k, r0 = divmod(n, 4)
    if r0 not in (0, 1) or k < 2:
        raise ValueError("Table 1 is used for n = 4k, 4k+1 with k >= 2")
    pairs: List[Tuple[int, int]] = []
    if r0 == 0:
        pairs += [(4 * k + r, 8 * k - r) for r in range(0, 2 * k)]
        pairs += [(2 * k + 1, 6 * k), (2 * k, 4 * k - 1)]
        pairs += [(r, 4 * k - 1 - r) for r in range(1, k)]
        pairs += [(k, k + 1)]
        pairs += [(k + 2 + r, 3 * k - 1 - r) for r in range(0, k - 2)]
    else:
        pairs += [(4 * k + 2 + r, 8 * k + 2 - r) for r in range(0, 2 * k)]
        pairs += [(2 * k + 1, 6 * k + 2), (2 * k + 2, 4 * k + 1)]
        pairs += [(r, 4 * k + 1 - r) for r in range(1, k + 1)]
        pairs += [(k + 1, k + 2)]
        pairs += [(k + 2 + r, 3 * k + 1 - r) for r in range(1, k - 1)]
    return sorted(pairs, key=lambda ab: ab[1] - ab[0])


def _run(a: int, b: int, step_down: bool) -> List[int]:
    """Table 2's "a, ..., b" in steps of 2; empty when a is already past b."""
    if step_down:
        return list(range(a, b - 1, -2)) if a >= b else []
    return list(range(a, b + 1, 2)) if a <= b else []


def davies_construction(n: int) -> List[int]:
    """Table 2 (Davies' construction): a Langford sequence (labels by position)
    for n = 4k - 1 and n = 4k, k >= 1."""
    if n % 4 == 3:
        k = (n + 1) // 4
        seq = (_run(4 * k - 4, 2 * k, True) + [4 * k - 2] + _run(2 * k - 3, 1, True) +
               [4 * k - 1] + _run(1, 2 * k - 3, False) + _run(2 * k, 4 * k - 4, False) +
               [2 * k - 1] + _run(4 * k - 3, 2 * k + 1, True) + [4 * k - 2] +
               _run(2 * k - 2, 2, True) + [2 * k - 1, 4 * k - 1] + _run(2, 2 * k - 2, False) +
               _run(2 * k + 1, 4 * k - 3, False))
    elif n % 4 == 0:
        k = n // 4
        seq = (_run(4 * k - 4, 2 * k, True) + [4 * k - 2] + _run(2 * k - 3, 1, True) +
               [4 * k - 1] + _run(1, 2 * k - 3, False) + _run(2 * k, 4 * k - 4, False) +
               [4 * k] + _run(4 * k - 3, 2 * k + 1, True) + [4 * k - 2] +
               _run(2 * k - 2, 2, True) + [2 * k - 1, 4 * k - 1] + _run(2, 2 * k - 2, False) +
               _run(2 * k + 1, 4 * k - 3, False) + [2 * k - 1, 4 * k])
    else:
        raise ValueError("Table 2 covers n = 4k - 1 and n = 4k")
    return seq


def sequence_to_pairs(seq: Sequence[int], n: int) -> Optional[List[Tuple[int, int]]]:
    """Positions of the two copies of each label 1..n (None if malformed)."""
    where: Dict[int, List[int]] = {}
    for i, lab in enumerate(seq, start=1):
        where.setdefault(lab, []).append(i)
    pairs = []
    for k in range(1, n + 1):
        w = where.get(k, [])
        if len(w) != 2:
            return None
        pairs.append((w[0], w[1]))
    return pairs


# --------------------------------------------------------------------------
# Primes (for choosing moduli in tests)
# --------------------------------------------------------------------------

def is_prime(x: int) -> bool:
    """Deterministic Miller-Rabin for x < 3.3e24 (first 13 prime bases)."""
    if x < 2:
        return False
    small = [2, 3, 5, 7, 11, 13, 17, 19, 23, 29, 31, 37, 41]
    for q in small:
        if x % q == 0:
            return x == q
    d, s = x - 1, 0
    while d % 2 == 0:
        d //= 2
        s += 1
    for a in small:
        y = pow(a, d, x)
        if y in (1, x - 1):
            continue
        for _ in range(s - 1):
            y = y * y % x
            if y == x - 1:
                break
        else:
            return False
    return True


def primes_below(bound: int, count: int) -> List[int]:
    out = []
    x = bound - 1
    while len(out) < count:
        if is_prime(x):
            out.append(x)
        x -= 1
    return out


# --------------------------------------------------------------------------
# Approximate counting (Sec. 3, Algorithm 2)
# --------------------------------------------------------------------------

def philox4x32_10(ctr: Sequence[int], key: Sequence[int]) -> List[int]:
    """Philox4x32-10 (Salmon et al., SC'11) of a 4-word counter and 2-word key."""
    c = (ctypes.c_uint32 * 4)(*ctr)
    k = (ctypes.c_uint32 * 2)(*key)
    o = (ctypes.c_uint32 * 4)()
    lib().orc_philox4x32_10(c, k, o)
    return [int(x) for x in o]


def placements(n: int, variant) -> List[int]:
    """L_k: number of placements (a, a + d_k) of pair k inside P."""
    pos, d = instance(n, variant)
    s = set(pos)
    return [sum(1 for a in pos if a + dk in s) for dk in d]


def z0(n: int, variant) -> int:
    """Z(0): number of configurations of the relaxed problem (Sec. 3)."""
    out = 1
    for x in placements(n, variant):
        out *= x
    return out


def energy_histogram(n: int, variant) -> List[int]:
    """Number of configurations of the relaxed problem with each energy E
    (E = number of empty bins), by enumeration (use Z(0) < ~1e8)."""
    pos, _ = instance(n, variant)
    top = pos[-1]
    h = (ctypes.c_uint64 * (top + 1))()
    if lib().orc_energy_histogram(n, _variant(variant), h) != 0:
        raise ValueError("bad instance")
    return [int(x) for x in h]


def pt_ladder(n: int, variant, betas: Sequence[float], iters: int, seed: int, ladder: int = 0,
              schedule: str = "sweep") -> Dict:
    """Runs one tempering ladder (Algorithm 2) and returns energy histograms
    per level, move/exchange acceptance counts and the final states."""
    pos, _ = instance(n, variant)
    top = pos[-1]
    M = len(betas)
    H = top + 1
    b = (ctypes.c_double * M)(*betas)
    hist = (ctypes.c_uint64 * (M * H))()
    mv = (ctypes.c_uint64 * M)()
    sa = (ctypes.c_uint64 * M)()
    stry = (ctypes.c_uint64 * M)()
    fa = (ctypes.c_int * (M * n))()
    fe = (ctypes.c_int * M)()
    sch = {"sweep": 0, "even_odd": 1}[schedule]
    rc = lib().orc_pt_ladder(n, _variant(variant), M, b, iters, seed, ladder, sch, hist, mv, sa, stry, fa, fe)
    if rc != 0:
        raise ValueError(f"orc_pt_ladder failed ({rc})")
    return {"hist": [[int(hist[j * H + e]) for e in range(H)] for j in range(M)],
            "move_accept": [int(x) for x in mv], "swap_accept": [int(x) for x in sa],
            "swap_try": [int(x) for x in stry],
            "final_a": [[int(fa[j * n + k]) for k in range(n)] for j in range(M)],
            "final_e": [int(x) for x in fe]}


def pt_ratios(hist: Sequence[Sequence[int]], betas: Sequence[float]) -> List[float]:
    """Ratio(j) of Algorithm 2 from energy histograms: the mean of
    exp(-(beta_{j+1} - beta_j) E) at level j; the last level's ratio is taken
    to beta = infinity, i.e. the fraction of samples with E = 0."""
    out = []
    M = len(betas)
    for j in range(M):
        tot = sum(hist[j])
        if j + 1 < M:
            db = betas[j + 1] - betas[j]
            out.append(sum(c * math.exp(-db * e) for e, c in enumerate(hist[j])) / tot)
        else:
            out.append(hist[j][0] / tot)
    return out


def pt_estimate(hist, betas, n: int, variant, ordered: bool = False) -> float:
    """Z(0) times the product of the ratios (Sec. 3, end of Algorithm 2); the
    first inverse temperature must be 0.  Reflections counted once unless
    ``ordered`` (the 1/2 of Table 6)."""
    if betas[0] != 0:
        raise ValueError("the ladder must start at beta = 0")
    ratios = pt_ratios(hist, betas)
    if min(ratios) <= 0:
        return 0.0
    v = math.exp(math.log(z0(n, variant)) + sum(math.log(r) for r in ratios))
    if not ordered and _variant(variant) != HOOKED and n > 1:
        v /= 2
    return v
