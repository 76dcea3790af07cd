"""Pins for the tempering oracle (Sec. 3, Algorithm 2) on the CPU.

Sources: the closed form Z(0) = (2n-1)!/(n-1)! and the estimator of Sec. 3;
Table 6's sample run for S(12); exact energy distributions by enumeration;
Philox4x32-10 known-answer vectors from its authors' reference implementation.
"""
import json
import math
import os

import pytest

import oracle as O

GOLD = os.path.join(os.path.dirname(__file__), "golden")


@pytest.fixture(scope="module", autouse=True)
def _built():
    O.build(force=False)


def test_philox_known_answers():
    # Random123 known-answer vectors for philox4x32 with 10 rounds.
    assert O.philox4x32_10([0, 0, 0, 0], [0, 0]) == [0x6627E8D5, 0xE169C58D, 0xBC57AC4C, 0x9B00DBD8]
    assert O.philox4x32_10([0xFFFFFFFF] * 4, [0xFFFFFFFF] * 2) == [0x408F276D, 0x41C83B0E, 0xA20BC7C6,
                                                                   0x6D5451FD]
    assert O.philox4x32_10([0x243F6A88, 0x85A308D3, 0x13198A2E, 0x03707344], [0xA4093822, 0x299F31D0]) == \
        [0xD16CFE09, 0x94FDCCEB, 0x5001E420, 0x24126EA1]


@pytest.mark.parametrize("variant", ["skolem", "langford", "hooked"])
def test_energy_zero_configurations_are_the_pairings(variant):
    for n in range(1, 7):
        h = O.energy_histogram(n, variant)
        assert sum(h) == O.z0(n, variant)
        assert h[0] == O.count_backtrack(n, variant)


def test_z0_closed_form_sec3():
    for n in range(1, 12):
        assert O.z0(n, "skolem") == math.factorial(2 * n - 1) // math.factorial(n - 1)


def test_estimator_formula_exact_with_exact_ratios():
    """With the exact energy distributions at each level the estimator of
    Algorithm 2 returns the exact count (telescoping product of Sec. 3)."""
    for variant, n in [("skolem", 5), ("langford", 4), ("hooked", 6), ("langford", 7)]:
        N = O.energy_histogram(n, variant)
        betas = [0.0, 0.4, 1.1, 2.5, 5.0]
        weights = [[c * math.exp(-b * e) for e, c in enumerate(N)] for b in betas]
        est = O.pt_estimate(weights, betas, n, variant, ordered=True)
        assert est == pytest.approx(N[0], rel=1e-12)


def test_table6_assembly():
    t6 = json.load(open(os.path.join(GOLD, "table6_pt_n12.json")))
    est = 0.5 * math.factorial(23) / math.factorial(11) * math.prod(t6["ratio"])
    assert abs(est - t6["estimate"]) < 1.0


@pytest.mark.parametrize("schedule", ["sweep", "even_odd"])
def test_ladder_samples_boltzmann_distribution(schedule):
    """Energy histograms of every level match exp(-beta E) N(E) / Z(beta)."""
    n, v = 5, "skolem"
    N = O.energy_histogram(n, v)
    betas = [0.0, 0.5, 1.0, 2.0, 4.0]
    r = O.pt_ladder(n, v, betas, 1 << 18, seed=12345, schedule=schedule)
    for j, b in enumerate(betas):
        w = [c * math.exp(-b * e) for e, c in enumerate(N)]
        z = sum(w)
        emp = r["hist"][j]
        tot = sum(emp)
        tv = 0.5 * sum(abs(emp[e] / tot - w[e] / z) for e in range(len(N)))
        assert tv < 0.015, (schedule, j, tv)
    assert all(t > 0 for t in r["swap_try"][: len(betas) - 1])


@pytest.mark.parametrize("variant,n", [("skolem", 5), ("skolem", 8), ("langford", 7), ("hooked", 7)])
def test_small_estimates_near_exact(variant, n):
    """Sec. 3.1 reports no error for n < 12: the mean over independent ladders
    is within four standard errors (and 3 %) of the exact count."""
    betas = [0.0] + [0.25 * 1.45 ** i for i in range(12)]
    ests = []
    for ladder in range(8):
        r = O.pt_ladder(n, variant, betas, 1 << 16, seed=99, ladder=ladder, schedule="even_odd")
        ests.append(O.pt_estimate(r["hist"], betas, n, variant, ordered=True))
    exact = O.count_backtrack(n, variant)
    mean = sum(ests) / len(ests)
    se = math.sqrt(sum((e - mean) ** 2 for e in ests) / (len(ests) - 1) / len(ests))
    assert abs(mean - exact) < max(4 * se, 0.01 * exact), (ests, exact)
    assert abs(mean / exact - 1) < 0.03 + 4 * se / exact


def test_table6_run_reproduced():
    """The S(12) run of Table 6 (same twelve inverse temperatures): mean
    energies per level and the estimate agree with the printed ones."""
    t6 = json.load(open(os.path.join(GOLD, "table6_pt_n12.json")))
    betas = t6["beta"]
    runs = [O.pt_ladder(12, "skolem", betas, 1 << 20, seed=2017, ladder=L, schedule="sweep") for L in range(4)]
    for j, want in enumerate(t6["mean_energy"]):
        h = [sum(r["hist"][j][e] for r in runs) for e in range(len(runs[0]["hist"][j]))]
        mean = sum(e * c for e, c in enumerate(h)) / sum(h)
        assert abs(mean - want) < 0.06 + 0.05 * want, (j, mean, want)
    ests = [O.pt_estimate(r["hist"], betas, 12, "skolem") for r in runs]
    mean = sum(ests) / len(ests)
    se = math.sqrt(sum((e - mean) ** 2 for e in ests) / (len(ests) - 1) / len(ests))
    assert abs(mean - t6["exact"]) < max(4 * se, 0.01 * t6["exact"]), (ests, t6["exact"])
    assert abs(mean / t6["exact"] - 1) < 0.05
