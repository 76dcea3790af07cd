"""Tempering with the learned proposal on the GPU.

The network is trained on the chains' own states by the library's forward and
backward kernels, then used as an extra Metropolis-Hastings move.  Each level
keeps exp(-beta E) as its law, so the estimator stays unbiased: the estimates
are checked against exact counts from the CPU oracle.  The gain of training is
measured as the rate of accepted moves that change the configuration.
"""
import sys

import numpy as np
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


TABLE6_BETAS = [0, 0.54, 1.1, 1.69, 2.33, 3, 3.73, 4.65, 5.82, 8.1, 16, 32]


def _learned(**kw):
    d = dict(hidden1=64, hidden2=64, first_level=0, plain_per_learned=8, train_iterations=4096, snapshots=4,
             train_steps=150, minibatch=256, lr=2e-3, init_seed=1)
    d.update(kw)
    return d


@pytest.mark.parametrize("variant,n", [("skolem", 8), ("hooked", 10)])
def test_learned_estimate_within_error_of_exact(variant, n):
    betas = [0.0] + [0.25 * 1.45 ** i for i in range(12)]
    _say("learned pt", variant, n)
    est, se, st = sk.approx(n, variant, betas, ladders=64, iterations=1 << 17, seed=99,
                            proposal=sk.PROPOSAL_LEARNED, learned=_learned(train_iterations=1 << 15))
    exact = O.reported(O.count_backtrack(n, variant, threads=8), n, variant)
    _say("  estimate", est, "+-", se, "exact", exact, "learned moves", st["learned_moves"],
         "accept", [round(x, 3) for x in st["learned_accept"]], "train loss", st["train_loss"])
    assert st["learned_moves"] == (1 << 17) // 8
    assert abs(est - exact) < max(4 * se, 0.005 * exact)
    assert st["train_ms"] > 0 and st["gpu_ms"] > st["train_ms"]


def test_learned_run_is_reproducible():
    betas = [0.0, 0.5, 1.5, 3.0, 6.0]
    kw = dict(ladders=8, iterations=1024, seed=5, proposal=sk.PROPOSAL_LEARNED,
              learned=_learned(train_iterations=256, train_steps=20, minibatch=64))
    a = sk.pt_run(9, "skolem", betas, **kw)
    b = sk.pt_run(9, "skolem", betas, **kw)
    assert a["hist"] == b["hist"] and a["state"] == b["state"] and a["energy"] == b["energy"]


def test_frozen_and_returned_networks():
    n, betas = 7, [0.0, 0.7, 2.0, 5.0]
    P = sk.mlp_init(n, "skolem", 32, 32, seed=3)
    P0 = P.copy()
    # train_steps > 0 with params given: the trained network is written back
    sk.approx(n, "skolem", betas, 16, 512, 1, proposal=sk.PROPOSAL_LEARNED,
              learned=_learned(hidden1=32, hidden2=32, params=P, train_iterations=128, train_steps=10, minibatch=32))
    assert not np.array_equal(P, P0)
    # train_steps = 0: the given network is used frozen and left as it is
    P1 = P.copy()
    est, se, st = sk.approx(n, "skolem", betas, 16, 512, 1, proposal=sk.PROPOSAL_LEARNED,
                            learned=_learned(hidden1=32, hidden2=32, params=P, train_steps=0))
    assert np.array_equal(P, P1) and st["train_ms"] == 0 and st["learned_moves"] == 512 // 8


def test_the_states_stay_valid_and_energies_match():
    betas = [0.0, 0.4, 1.2, 3.0, 8.0]
    n = 10
    r = sk.pt_run(n, "langford", betas, 4, 999, 17, proposal=sk.PROPOSAL_LEARNED,
                  learned=_learned(train_iterations=200, train_steps=10, minibatch=64, plain_per_learned=3))
    pos, d = O.instance(n, "langford")
    for lad in range(4):
        for j in range(len(betas)):
            a = r["state"][lad][j]
            occ = {}
            for k in range(n):
                assert a[k] in pos and a[k] + d[k] in pos
                occ[a[k]] = occ.get(a[k], 0) + 1
                occ[a[k] + d[k]] = occ.get(a[k] + d[k], 0) + 1
            assert r["energy"][lad][j] == sum(1 for p in pos if p not in occ)
    assert sum(sum(sum(h) for h in lad) for lad in r["hist"]) == 4 * len(betas) * 999


def test_training_gains_over_untrained_network():
    """Rate of accepted configuration-changing learned moves, trained network
    against the same network untrained (Table 6's S(12) ladder)."""
    n = 12
    common = dict(ladders=64, iterations=1 << 16, seed=2024, proposal=sk.PROPOSAL_LEARNED)
    P = sk.mlp_init(n, "skolem", 128, 128, seed=8)
    est0, se0, st0 = sk.approx(n, "skolem", TABLE6_BETAS, **common,
                               learned=_learned(hidden1=128, hidden2=128, params=P.copy(), train_steps=0,
                                                train_iterations=1 << 14))
    est1, se1, st1 = sk.approx(n, "skolem", TABLE6_BETAS, **common,
                               learned=_learned(hidden1=128, hidden2=128, params=P, train_iterations=1 << 14,
                                                snapshots=8, train_steps=600, minibatch=512))
    plain = sk.approx(n, "skolem", TABLE6_BETAS, ladders=64, iterations=1 << 16, seed=2024,
                      burn_in=1 << 14)[2]
    _say("untrained accept", [round(x, 3) for x in st0["learned_accept"]])
    _say("trained   accept", [round(x, 3) for x in st1["learned_accept"]], "loss", st1["train_loss"])
    _say("plain move accept", [round(x, 3) for x in plain["move_accept"]])
    _say("estimates", est0, se0, est1, se1, "exact 227968")
    mid = range(2, len(TABLE6_BETAS) - 3)
    assert sum(st1["learned_accept"][j] for j in mid) > 1.5 * sum(st0["learned_accept"][j] for j in mid)
    for est, se in ((est0, se0), (est1, se1)):
        assert abs(est - 227968) < max(4 * se, 0.01 * 227968)


def test_invalid_learned_parameters():
    betas = [0.0, 1.0]
    bad = [dict(first_level=2), dict(plain_per_learned=0), dict(train_steps=5, snapshots=0),
           dict(train_steps=5, lr=0.0), dict(train_steps=0)]  # a fresh network must be trained
    for kw in bad:
        with pytest.raises(sk.SkolemError):
            sk.approx(6, "skolem", betas, 2, 16, 1, proposal=sk.PROPOSAL_LEARNED, learned=_learned(**kw))
    with pytest.raises(sk.SkolemError):
        sk.approx(6, "skolem", betas, 2, 16, 1, proposal=sk.PROPOSAL_LEARNED, learned=None)


def test_learned_against_plain_tempering():
    """What the learned proposal gains and loses against plain tempering (the
    method without it: uniform moves, Sec. 3) on Table 6's S(12) ladder, at
    the same recorded iterations and seed.  Gains: at the middle levels the
    learned moves that change the configuration are accepted more often than
    the uniform moves there (on average over those levels), and the estimate's
    standard error is smaller.  Loss: the GPU time, since a learned move costs
    two network evaluations per chain where a uniform move costs a few
    instructions.  Both estimates are within error of the exact count."""
    n = 12
    it = 1 << 16
    plain_est, plain_se, plain = sk.approx(n, "skolem", TABLE6_BETAS, ladders=128, iterations=it, seed=77,
                                           burn_in=1 << 14)
    est, se, st = sk.approx(n, "skolem", TABLE6_BETAS, ladders=128, iterations=it, seed=77,
                            proposal=sk.PROPOSAL_LEARNED,
                            learned=_learned(hidden1=128, hidden2=128, train_iterations=1 << 14, snapshots=8,
                                             train_steps=600, minibatch=512))
    mid = list(range(2, len(TABLE6_BETAS) - 3))
    gain = [st["learned_accept"][j] / plain["move_accept"][j] for j in mid]
    _say("learned/plain acceptance at the middle levels", [round(g, 2) for g in gain])
    _say("GPU s: plain", plain["gpu_ms"] / 1e3, "learned", st["gpu_ms"] / 1e3,
         "standard errors", plain_se, se, "estimates", plain_est, est)
    assert sum(gain) / len(gain) > 1.2
    assert se < plain_se
    assert st["gpu_ms"] > 2 * plain["gpu_ms"]
    for e, s in ((plain_est, plain_se), (est, se)):
        assert abs(e - 227968) < max(4 * s, 0.01 * 227968)
