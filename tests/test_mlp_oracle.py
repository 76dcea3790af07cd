"""Pins for the learned-proposal oracle (oracle/mlp.py): gradient against
finite differences, the heat-bath target against enumeration, and the
Metropolis-Hastings correction against the exact Boltzmann distribution."""
import math
import random

import numpy as np
import pytest

import oracle as O
from oracle import mlp


def test_feature_width_matches_the_configured_network():
    g = mlp.Geometry(32, "skolem")
    assert g.din == 130 and g.dout == 32 * 64


def test_features_definition():
    g = mlp.Geometry(4, "skolem")
    a = [7, 3, 1, 2]  # pairs (7,8) (3,5) (1,4) (2,6): a Skolem pairing
    x = mlp.features(g, a, 1.5)
    assert list(x[:8]) == [1.0] * 8
    assert list(x[8:12]) == [7 / 8, 3 / 8, 1 / 8, 2 / 8]
    assert list(x[12:16]) == [0.0] * 4 and x[16] == 1.5 and x[17] == 0.0
    b = [1, 3, 1, 2]  # pair 1 moved onto pair 3's first bin
    y = mlp.features(g, b, 0.0)
    assert y[12] == 1.0 and y[14] == 1.0 and y[17] == g.energy(b) / 8 > 0


def test_gradient_against_finite_differences():
    g = mlp.Geometry(4, "langford")
    P = mlp.init_params(g, h1=7, h2=5, seed=3, scale=1.5)
    rng = random.Random(5)
    states = [[rng.choice([a for a in range(1, g.T + 1) if g.valid[k, a - 1]]) for k in range(g.n)]
              for _ in range(6)]
    betas = [0.0, 0.3, 1.0, 2.0, 0.7, 3.0]
    loss, G = mlp.loss_and_grad(P, g, states, betas)
    h = 1e-6
    for name in ("W1", "b1", "W2", "b2", "W3", "b3"):
        flat = P[name].reshape(-1)
        for idx in list(range(0, flat.size, max(1, flat.size // 7)))[:7]:
            old = flat[idx]
            flat[idx] = old + h
            lp, _ = mlp.loss_and_grad(P, g, states, betas)
            flat[idx] = old - h
            lm, _ = mlp.loss_and_grad(P, g, states, betas)
            flat[idx] = old
            num = (lp - lm) / (2 * h)
            ana = G[name].reshape(-1)[idx]
            assert abs(num - ana) <= 1e-6 + 1e-5 * abs(num), (name, idx, num, ana)


def test_target_is_heat_bath_over_single_pair_moves():
    g = mlp.Geometry(5, "skolem")
    a = [1, 2, 3, 4, 5]
    beta = 0.8
    t = mlp.target(g, a, beta)
    assert abs(t.sum() - 1) < 1e-12
    assert np.all(t[~g.valid.reshape(-1)] == 0)
    # ratio of two entries equals the Boltzmann factor of their energies
    b1 = list(a); b1[0] = 8
    b2 = list(a); b2[3] = 2
    r = t[0 * g.T + 7] / t[3 * g.T + 1]
    assert r == pytest.approx(math.exp(-beta * (g.energy(b1) - g.energy(b2))), rel=1e-12)


def test_adam_matches_definition():
    P = {"w": np.array([1.0, -2.0])}
    G = {"w": np.array([0.5, 0.25])}
    M = {"w": np.zeros(2)}
    V = {"w": np.zeros(2)}
    mlp.adam(P, G, M, V, 1, lr=0.1)
    # first step: m_hat = g, v_hat = g^2 -> step = lr * sign(g)
    assert P["w"] == pytest.approx([1.0 - 0.1, -2.0 - 0.1], rel=1e-6)


@pytest.mark.parametrize("beta", [0.0, 1.5])
def test_learned_proposal_chain_is_exact(beta):
    """With arbitrary (random) weights the corrected chain samples
    exp(-beta E) over all configurations: energy histogram vs enumeration."""
    n, v = 4, "skolem"
    g = mlp.Geometry(n, v)
    P = mlp.init_params(g, h1=16, h2=16, seed=11, scale=1.0)
    N = O.energy_histogram(n, v)
    w = [c * math.exp(-beta * e) for e, c in enumerate(N)]
    z = sum(w)
    rng = random.Random(17)
    a = [int(np.flatnonzero(g.valid[k])[0]) + 1 for k in range(n)]
    hist = [0] * len(N)
    steps = 40000
    for _ in range(steps):
        a, _ok = mlp.mh_learned_step(P, g, a, beta, rng.random(), rng.random())
        hist[g.energy(a)] += 1
    tv = 0.5 * sum(abs(hist[e] / steps - w[e] / z) for e in range(len(N)))
    # dropping the q-ratio gives 0.018 (beta 0) and 0.053 (beta 1.5) here
    assert tv < (0.01 if beta == 0 else 0.025), (tv, hist)
