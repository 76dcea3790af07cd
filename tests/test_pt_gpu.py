"""GPU tempering (Sec. 3, Algorithm 2) against the CPU oracle.

The chains use the same Philox4x32-10 streams and the same integer accept
thresholds on both sides, so histograms, acceptance counts and final states
must agree bit for bit (oracle schedule "even_odd").  The estimator is then
checked statistically against exact counts.
"""
import math
import sys

import pytest

import oracle as O
import paper_1507_00315_amd as sk

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module", autouse=True)
def _ready():
    O.build(force=False)
    sk.lib()


CASES = [("skolem", 5, [0.0, 0.3, 0.8, 1.5, 3.0, 6.0]),
         ("skolem", 8, [0.0, 0.5, 1.0, 2.0, 4.0]),
         ("langford", 7, [0.0, 0.4, 1.2, 2.5, 5.0, 9.0, 14.0]),
         ("hooked", 7, [0.0, 0.7, 2.0, 4.0]),
         ("skolem", 12, [0.0, 0.54, 1.1, 1.69, 2.33, 3, 3.73, 4.65, 5.82, 8.1, 16, 32])]


@pytest.mark.parametrize("variant,n,betas", CASES)
def test_chains_bit_exact_against_oracle(variant, n, betas):
    ladders, iters, seed = 3, 4000, 777 + n
    g = sk.pt_run(n, variant, betas, ladders, iters, seed)
    for lad in range(ladders):
        _say("pt parity", variant, n, "ladder", lad)
        o = O.pt_ladder(n, variant, betas, iters, seed, ladder=lad, schedule="even_odd")
        assert g["hist"][lad] == o["hist"]
        assert g["move_accept"][lad] == o["move_accept"]
        assert g["swap_accept"][lad][: len(betas) - 1] == o["swap_accept"][: len(betas) - 1]
        assert g["state"][lad] == o["final_a"]
        assert g["energy"][lad] == o["final_e"]


def test_segments_carry_the_chains():
    """Several kernel launches (segments) continue the same chains."""
    betas = [0.0, 0.5, 1.5, 3.0, 6.0]
    a = sk.pt_run(9, "skolem", betas, 2, 5000, 31, segment=777)
    o = O.pt_ladder(9, "skolem", betas, 5000, 31, ladder=1, schedule="even_odd")
    assert a["hist"][1] == o["hist"] and a["state"][1] == o["final_a"]


@pytest.mark.parametrize("variant,segment", [("skolem", 1), ("langford", 2), ("skolem", 63), ("hooked", 64),
                                             ("skolem", 65)])
def test_segment_lengths_around_the_philox_groups(variant, segment):
    """The kernel draws the wave-shared parts of the Philox blocks for 64
    block numbers at a time: launches of any length (one iteration, fewer than
    64, exactly 64, one more), starting anywhere inside such a group, continue
    the same chains as the oracle's single run."""
    betas = [0.0, 0.5, 1.5, 3.0, 6.0]
    iters, seed = 200, 4242
    _say("pt segments", variant, segment)
    g = sk.pt_run(9, variant, betas, 2, iters, seed, segment=segment)
    for lad in range(2):
        o = O.pt_ladder(9, variant, betas, iters, seed, ladder=lad, schedule="even_odd")
        assert g["hist"][lad] == o["hist"]
        assert g["move_accept"][lad] == o["move_accept"]
        assert g["state"][lad] == o["final_a"] and g["energy"][lad] == o["final_e"]


def test_max_levels_and_size():
    betas = [0.0] + [0.05 * (120 ** (j / 62)) for j in range(63)]
    g = sk.pt_run(32, "skolem", betas, 1, 300, 5)
    o = O.pt_ladder(32, "skolem", betas, 300, 5, ladder=0, schedule="even_odd")
    assert g["hist"][0] == o["hist"] and g["state"][0] == o["final_a"]


@pytest.mark.parametrize("variant,n", [("skolem", 8), ("langford", 8), ("hooked", 10)])
def test_estimate_within_error_of_exact(variant, n):
    # Recording from the first iteration (as Algorithm 2 is printed) biases
    # short runs low: every ladder starts far from equilibrium at its top
    # levels, so the bias is common to all ladders and invisible in their
    # spread (the oracle shows z = -4.5 for Langford n = 8 at 2^15
    # iterations).  A burn-in of 2^15 iterations removes it (|z| < 1 there).
    betas = [0.0] + [0.25 * 1.45 ** i for i in range(12)]
    est, se, st = sk.approx(n, variant, betas, ladders=64, iterations=1 << 18, seed=4242, burn_in=1 << 15)
    exact = O.reported(O.count_backtrack(n, variant, threads=8), n, variant)
    _say(variant, n, est, se, exact)
    assert abs(est - exact) < max(4 * se, 0.005 * exact)
    assert 0 < st["move_accept"][0] <= 1 and st["gpu_ms"] > 0
    assert st["moves"] == 64 * len(betas) * (1 << 18)


def test_invalid_ladders():
    with pytest.raises(sk.SkolemError):
        sk.approx(8, "skolem", [0.1, 0.5], 1, 10, 1)   # must start at beta = 0
    with pytest.raises(sk.SkolemError):
        sk.approx(8, "skolem", [0.0, 0.5, 0.4], 1, 10, 1)  # not ascending
    with pytest.raises(sk.SkolemError):
        sk.approx(1, "langford", [0.0, 1.0], 1, 10, 1)  # no configuration


def test_burn_in_is_not_recorded_and_continues_the_chains():
    """burn_in b then i recorded iterations equals the last i iterations of an
    unburnt run of b + i (same Philox counters): histograms differ by the
    first b iterations' histogram."""
    betas = [0.0, 0.5, 1.5, 3.0, 6.0]
    full = sk.pt_run(9, "skolem", betas, 2, 3000, 31)
    head = sk.pt_run(9, "skolem", betas, 2, 1000, 31)
    tail = sk.pt_run(9, "skolem", betas, 2, 2000, 31, burn_in=1000)
    for lad in range(2):
        for j in range(len(betas)):
            assert [a - b for a, b in zip(full["hist"][lad][j], head["hist"][lad][j])] == tail["hist"][lad][j]
        assert tail["state"][lad] == full["state"][lad] and tail["energy"][lad] == full["energy"][lad]


@pytest.mark.parametrize("variant,n", [("skolem", 33), ("langford", 32), ("hooked", 40)])
def test_chains_bit_exact_beyond_64_positions(variant, n):
    """Instances with more than 64 positions (S(33) of Table 7 among them)
    run the same chains as the oracle."""
    betas = [0.0] + [0.05 * 120 ** (j / 15) for j in range(16)]
    g = sk.pt_run(n, variant, betas, 2, 1500, 99)
    for lad in range(2):
        o = O.pt_ladder(n, variant, betas, 1500, 99, ladder=lad, schedule="even_odd")
        assert g["hist"][lad] == o["hist"] and g["state"][lad] == o["final_a"]
        assert g["energy"][lad] == o["final_e"]


def test_half_split_flags_unequilibrated_runs():
    """The two halves of a run: an equilibrated run (burn-in, many
    iterations) gives halves within their errors; a short run recorded from
    the first iteration (as Algorithm 2 is printed) on a large instance gives
    a first half biased low, flagged by half_z."""
    betas = [0.0] + [0.25 * 1.45 ** i for i in range(12)]
    est, se, st = sk.approx(12, "skolem", betas, ladders=64, iterations=1 << 17, seed=11, burn_in=1 << 15)
    _say("equilibrated halves", st["estimate_half"], st["std_error_half"], st["half_z"])
    assert abs(st["half_z"]) < 4
    assert all(abs(h - 227968) < 6 * e for h, e in zip(st["estimate_half"], st["std_error_half"]))
    ladder = [0.0] + [0.05 * 120.0 ** (j / 47) for j in range(48)]
    est, se, st = sk.approx(24, "skolem", ladder, ladders=256, iterations=1 << 12, seed=12)
    _say("short run halves", st["estimate_half"], st["std_error_half"], st["half_z"], est, se)
    assert st["half_z"] > 3 and st["estimate_half"][0] < st["estimate_half"][1]


def test_tuned_ladder_meets_the_exchange_target():
    """Sec. 3: exchanges of neighbouring levels accepted at least half the
    time, with a limited number of levels; the tuned ladder then estimates
    S(13) and L(12) within error."""
    for variant, n in (("skolem", 13), ("langford", 12)):
        betas, acc = sk.pt_tune_ladder(n, variant, 8.0, target=0.5, max_levels=64, ladders=128,
                                       pilot_iterations=1 << 13, seed=5)
        _say("tuned ladder", variant, n, len(betas), [round(b, 3) for b in betas], [round(a, 2) for a in acc])
        assert betas[0] == 0.0 and betas[-1] == 8.0 and all(b > a for a, b in zip(betas, betas[1:]))
        assert len(betas) < 64 and min(acc) >= 0.5
        est, se, st = sk.approx(n, variant, betas, ladders=128, iterations=1 << 17, seed=21, burn_in=1 << 15)
        exact = O.reported(O.count_backtrack(n, variant, threads=8), n, variant)
        _say("  estimate", est, se, exact, "min swap accept", min(st["swap_accept"][:len(betas) - 1]))
        assert abs(est - exact) < max(4 * se, 0.01 * exact)
