"""CPU oracle (float64, numpy) for the learned proposal of the tempering path.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

The paper's chains (Sec. 3) move one pair to a uniformly random placement.  The
learned proposal replaces that draw by a distribution q(k, a' | C) over every
(pair k, placement a') computed by a small MLP from the configuration C, and
keeps the chain exact with the Metropolis-Hastings acceptance

    min(1, exp(-beta (E(C') - E(C))) * q(k, a_k | C') / q(k, a' | C)),

C' being C with pair k moved to a'.  It is trained on chain states to match
the heat-bath distribution over single-pair moves,

    p*(k, a' | C)  proportional to  exp(-beta E(C with a_k = a')),

by minimising the cross-entropy -sum p* log q.  Everything below is written
from these definitions:

* features(C, beta): occupancy indicator of each bin (T values), a_k / T (n),
  1 if pair k shares a bin with another ball (n), beta, E / (2n); for n = 32
  Skolem that is 64 + 32 + 32 + 2 = 130 inputs.
* MLP: h1 = relu(W1 x + b1), h2 = relu(W2 h1 + b2), z = W3 h2 + b3, with z
  indexed by k * T + (a' - 1); entries of impossible placements are masked.
* loss_and_grad: mean cross-entropy over a batch and its exact gradient
  (checked against finite differences in tests/test_mlp_oracle.py).
* adam: one Adam step (Kingma and Ba, 2015).
"""
from __future__ import annotations

import math
from typing import Dict, List, Sequence, Tuple

import numpy as np

from . import instance, _variant


class Geometry:
    """Bins 1..T, the position set, differences and valid placements."""

    def __init__(self, n: int, variant):
        pos, d = instance(n, variant)
        self.n = n
        self.variant = _variant(variant)
        self.T = pos[-1]
        self.m = len(pos)
        self.pset = set(pos)
        self.d = d
        self.valid = np.zeros((n, self.T), dtype=bool)
        for k, dk in enumerate(d):
            for a in pos:
                if a + dk in self.pset:
                    self.valid[k, a - 1] = True
        self.din = self.T + 2 * n + 2
        self.dout = n * self.T

    def occupancy(self, a: Sequence[int]) -> np.ndarray:
        occ = np.zeros(self.T + 1, dtype=np.int64)
        for k, ak in enumerate(a):
            occ[ak] += 1
            occ[ak + self.d[k]] += 1
        return occ

    def energy(self, a: Sequence[int]) -> int:
        occ = self.occupancy(a)
        return sum(1 for p in self.pset if occ[p] == 0)


def features(g: Geometry, a: Sequence[int], beta: float) -> np.ndarray:
    occ = g.occupancy(a)
    x = np.zeros(g.din)
    for p in range(1, g.T + 1):
        x[p - 1] = 1.0 if occ[p] > 0 else 0.0
    for k, ak in enumerate(a):
        x[g.T + k] = ak / g.T
        x[g.T + g.n + k] = 1.0 if (occ[ak] > 1 or occ[ak + g.d[k]] > 1) else 0.0
    x[g.T + 2 * g.n] = beta
    x[g.T + 2 * g.n + 1] = g.energy(a) / g.m
    return x


def init_params(g: Geometry, h1: int = 256, h2: int = 256, seed: int = 0, scale: float = 1.0) -> Dict:
    rng = np.random.default_rng(seed)
    return {"W1": rng.standard_normal((h1, g.din)) * scale / math.sqrt(g.din), "b1": np.zeros(h1),
            "W2": rng.standard_normal((h2, h1)) * scale / math.sqrt(h1), "b2": np.zeros(h2),
            "W3": rng.standard_normal((g.dout, h2)) * scale / math.sqrt(h2), "b3": np.zeros(g.dout)}


def forward(P: Dict, X: np.ndarray) -> Tuple[np.ndarray, Dict]:
    """X: (B, din) -> logits (B, dout) and the activations needed backward."""
    a1 = X @ P["W1"].T + P["b1"]
    h1 = np.maximum(a1, 0.0)
    a2 = h1 @ P["W2"].T + P["b2"]
    h2 = np.maximum(a2, 0.0)
    z = h2 @ P["W3"].T + P["b3"]
    return z, {"X": X, "a1": a1, "h1": h1, "a2": a2, "h2": h2}


def masked_log_softmax(z: np.ndarray, mask: np.ndarray) -> np.ndarray:
    """log q over the entries where mask is True (-inf elsewhere); z: (..., dout)."""
    zm = np.where(mask, z, -np.inf)
    mx = np.max(zm, axis=-1, keepdims=True)
    lse = mx + np.log(np.sum(np.exp(zm - mx), axis=-1, keepdims=True))
    return zm - lse


def target(g: Geometry, a: Sequence[int], beta: float) -> np.ndarray:
    """p*(k, a') proportional to exp(-beta E(C with a_k = a')) over valid moves."""
    out = np.zeros(g.dout)
    es = []
    for k in range(g.n):
        for ap in range(1, g.T + 1):
            if g.valid[k, ap - 1]:
                b = list(a)
                b[k] = ap
                es.append((k * g.T + ap - 1, g.energy(b)))
    e0 = min(e for _, e in es)
    for idx, e in es:
        out[idx] = math.exp(-beta * (e - e0))
    return out / out.sum()


def loss_and_grad(P: Dict, g: Geometry, states: List[Sequence[int]], betas: Sequence[float]):
    """Mean over the batch of -sum_j p*_j log q_j, and its gradient."""
    X = np.stack([features(g, a, b) for a, b in zip(states, betas)])
    Tg = np.stack([target(g, a, b) for a, b in zip(states, betas)])
    mask = np.broadcast_to(g.valid.reshape(-1), (len(states), g.dout))
    z, c = forward(P, X)
    lq = masked_log_softmax(z, mask)
    B = len(states)
    loss = -np.sum(np.where(mask, Tg * lq, 0.0)) / B
    q = np.where(mask, np.exp(lq), 0.0)
    dz = (q - Tg) / B
    grads = {"W3": dz.T @ c["h2"], "b3": dz.sum(0)}
    dh2 = dz @ P["W3"]
    da2 = dh2 * (c["a2"] > 0)
    grads["W2"] = da2.T @ c["h1"]
    grads["b2"] = da2.sum(0)
    dh1 = da2 @ P["W2"]
    da1 = dh1 * (c["a1"] > 0)
    grads["W1"] = da1.T @ c["X"]
    grads["b1"] = da1.sum(0)
    return loss, grads


def adam(P: Dict, G: Dict, M: Dict, V: Dict, t: int, lr: float = 1e-3, b1: float = 0.9, b2: float = 0.999,
         eps: float = 1e-8) -> None:
    """One Adam step in place (t counts from 1)."""
    for k in P:
        M[k] = b1 * M[k] + (1 - b1) * G[k]
        V[k] = b2 * V[k] + (1 - b2) * G[k] * G[k]
        mh = M[k] / (1 - b1 ** t)
        vh = V[k] / (1 - b2 ** t)
        P[k] = P[k] - lr * mh / (np.sqrt(vh) + eps)


def mh_learned_step(P: Dict, g: Geometry, a: List[int], beta: float, u_pick: float, u_acc: float):
    """One Metropolis-Hastings step with the learned proposal.  u_pick picks
    (k, a') by inverting the cumulative distribution of q; u_acc decides.
    Returns (new state, accepted)."""
    mask = g.valid.reshape(-1)
    z, _ = forward(P, features(g, a, beta)[None, :])
    lq = masked_log_softmax(z, mask[None, :])[0]
    q = np.exp(lq)
    cdf = np.cumsum(np.where(mask, q, 0.0))
    j = int(np.searchsorted(cdf, u_pick * cdf[-1], side="right"))
    j = min(j, g.dout - 1)
    while not mask[j]:
        j -= 1
    k, ap = divmod(j, g.T)
    ap += 1
    b = list(a)
    old = b[k]
    b[k] = ap
    zb, _ = forward(P, features(g, b, beta)[None, :])
    lqb = masked_log_softmax(zb, mask[None, :])[0]
    log_alpha = -beta * (g.energy(b) - g.energy(a)) + lqb[k * g.T + old - 1] - lq[j]
    if math.log(max(u_acc, 1e-300)) < min(0.0, log_alpha):
        return b, True
    return a, False
