"""GPU proposal network against the float64 CPU oracle (oracle/mlp.py).

The network runs in fp32 (MFMA GEMMs, wave-level softmax); the oracle in
fp64.  Forward logits, loss and gradients are compared with tolerances derived
from fp32 rounding over the contraction lengths used here (relative error of a
length-K fp32 dot product is at most about K * 2^-24; K <= 2048 here, and the
observed errors sit far below the bounds).  Integer decisions (which move is
proposed, whether it is accepted) are compared where the oracle's fp64 margin
exceeds the fp32 error; the rest are checked for validity.  Exactness in
distribution of the Metropolis-Hastings move is checked against the exact
Boltzmann law of a small instance, enumerated on the host.
"""
import itertools
import math
import sys

import numpy as np
import pytest

import oracle as O
from oracle import mlp as OM
import paper_1507_00315_amd as sk

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module", autouse=True)
def _ready():
    O.build(force=False)
    sk.lib()


def unpack(g: OM.Geometry, P: np.ndarray, h1: int, h2: int):
    """Flat fp32 parameters (W1 b1 W2 b2 W3 b3, row-major) -> oracle dict (fp64)."""
    P = P.astype(np.float64)
    out, o = {}, 0
    for name, shape in (("W1", (h1, g.din)), ("b1", (h1,)), ("W2", (h2, h1)), ("b2", (h2,)),
                        ("W3", (g.dout, h2)), ("b3", (g.dout,))):
        size = int(np.prod(shape))
        out[name] = P[o:o + size].reshape(shape)
        o += size
    assert o == P.size
    return out


def pack(d) -> np.ndarray:
    return np.concatenate([d[k].reshape(-1) for k in ("W1", "b1", "W2", "b2", "W3", "b3")]).astype(np.float32)


def random_states(g: OM.Geometry, B: int, rng) -> np.ndarray:
    S = np.zeros((B, g.n), dtype=np.uint8)
    for k in range(g.n):
        choices = np.nonzero(g.valid[k])[0] + 1
        S[:, k] = rng.choice(choices, size=B)
    return S


SHAPES = [  # (variant, n, h1, h2, batch): ragged tiles in every GEMM dimension
    ("skolem", 6, 80, 48, 100),
    ("langford", 7, 64, 72, 37),
    ("hooked", 5, 33, 65, 129),
    ("skolem", 32, 256, 256, 70),   # the full-size network (130 -> 256 -> 256 -> 2048)
    ("langford", 6, 96, 64, 1024),  # long batch: weight gradients split along K
]


@pytest.mark.parametrize("variant,n,h1,h2,B", SHAPES)
def test_forward_matches_oracle(variant, n, h1, h2, B):
    _say("mlp forward", variant, n, h1, h2, B)
    g = OM.Geometry(n, variant)
    rng = np.random.default_rng(11 + n)
    P = sk.mlp_init(n, variant, h1, h2, seed=3, scale=1.5)
    S = random_states(g, B, rng)
    betas = rng.uniform(0, 6, size=B)
    z = sk.mlp_forward(n, variant, P, S, betas, h1, h2)
    X = np.stack([OM.features(g, list(S[i]), betas[i]) for i in range(B)])
    zo, _ = OM.forward(unpack(g, P, h1, h2), X)
    scale = np.abs(zo).max()
    err = np.abs(z - zo).max()
    _say("  max |dz| =", err, "max |z| =", scale)
    assert err <= 2e-5 * max(scale, 1.0) * math.sqrt(max(h1, h2, g.din))


def test_forward_large_batch_matches_oracle():
    """A batch large enough for the 128 x 128-tile product (at least 1024
    output tiles with both operands contiguous along k: the last layer over
    8256 states, a ragged last row tile) against the fp64 oracle."""
    variant, n, h1, h2, B = "skolem", 32, 256, 256, 8256
    _say("mlp forward, large batch", variant, n, h1, h2, B)
    g = OM.Geometry(n, variant)
    rng = np.random.default_rng(47)
    P = sk.mlp_init(n, variant, h1, h2, seed=9, scale=1.5)
    S = random_states(g, B, rng)
    betas = rng.uniform(0, 6, size=B)
    z = sk.mlp_forward(n, variant, P, S, betas, h1, h2)
    X = np.stack([OM.features(g, list(S[i]), betas[i]) for i in range(B)])
    zo, _ = OM.forward(unpack(g, P, h1, h2), X)
    scale = np.abs(zo).max()
    err = np.abs(z - zo).max()
    _say("  max |dz| =", err, "max |z| =", scale)
    assert err <= 2e-5 * max(scale, 1.0) * math.sqrt(max(h1, h2, g.din))


U32 = 2.0 ** -24  # unit roundoff of fp32


def grad_error_bound(Pd, g: OM.Geometry, states, betas, lam=None):
    """Element-wise bound on the fp32 gradient's distance from the fp64 one.

    The gradient is a chain of dot products (backward through three layers,
    each a sum over the batch).  A length-K fp32 dot product has error at most
    K u sum |x_i y_i| (u = 2^-24; the worst case, lam=None), or with
    probability at least 1 - 2 exp(-lam^2 / 2) at most lam sqrt(K) u sum |x_i y_i|
    when the rounding errors are independent (Higham and Mary, SIAM J. Sci.
    Comput. 2019; lam=6).  Errors already in a product's inputs enter the same
    sum of absolute products.  So every gradient entry is bounded by
    c e(K_chain) M, where M is the same backward pass run on absolute values
    (|W|, |h|, and |dz| replaced by (q + p*) / B, which bounds dz = (q - p*) / B,
    with q widened by the relative change the logits' own fp32 error causes),
    K_chain the sum of the contraction lengths on the path plus the forward
    pass's, and ReLU masks widened to pre-activations within the forward
    error of zero, where fp32 may take the other branch.
    Returns {name: bound array}."""
    def e(K):
        return K * U32 if lam is None else lam * math.sqrt(K) * U32

    X = np.stack([OM.features(g, list(a), b) for a, b in zip(states, betas)])
    Tg = np.stack([OM.target(g, list(a), b) for a, b in zip(states, betas)])
    mask = np.broadcast_to(g.valid.reshape(-1), (len(states), g.dout))
    z, c = OM.forward(Pd, X)
    q = np.where(mask, np.exp(OM.masked_log_softmax(z, mask)), 0.0)
    B = len(states)
    h1, h2 = Pd["W1"].shape[0], Pd["W2"].shape[0]
    A = {k: np.abs(v) for k, v in Pd.items()}
    a1_abs = np.abs(X) @ A["W1"].T + A["b1"]
    a2_abs = np.maximum(a1_abs, 0) @ A["W2"].T + A["b2"]
    z_abs = np.maximum(a2_abs, 0) @ A["W3"].T + A["b3"]
    k_fwd = g.din + h1 + h2
    k_chain = B + g.dout + h2 + h1 + k_fwd
    # the logits' error (per state, the largest) moves q by at most twice it, relative to q
    zq = 2 * e(k_fwd) * z_abs.max(axis=1, keepdims=True)
    dzA = (q * (1 + zq / e(k_chain)) + Tg) / B
    w1 = c["a1"] > -2 * e(k_fwd) * a1_abs
    w2 = c["a2"] > -2 * e(k_fwd) * a2_abs
    M = {"W3": dzA.T @ np.abs(c["h2"]), "b3": dzA.sum(0)}
    d2 = (dzA @ A["W3"]) * w2
    M["W2"] = d2.T @ np.abs(c["h1"])
    M["b2"] = d2.sum(0)
    d1 = (d2 @ A["W2"]) * w1
    M["W1"] = d1.T @ np.abs(X)
    M["b1"] = d1.sum(0)
    return {k: 4 * e(k_chain) * v for k, v in M.items()}


@pytest.mark.parametrize("variant,n,h1,h2,B", SHAPES)
def test_loss_and_gradient_match_oracle(variant, n, h1, h2, B):
    """Loss and every gradient entry against the fp64 oracle, each entry
    within the bound of grad_error_bound."""
    _say("mlp grad", variant, n, h1, h2, B)
    g = OM.Geometry(n, variant)
    rng = np.random.default_rng(21 + n)
    P = sk.mlp_init(n, variant, h1, h2, seed=5, scale=1.0)
    S = random_states(g, B, rng)
    betas = rng.uniform(0, 4, size=B)
    loss, grad = sk.mlp_loss_grad(n, variant, P, S, betas, h1, h2)
    Pd = unpack(g, P, h1, h2)
    lo, go = OM.loss_and_grad(Pd, g, [list(s) for s in S], list(betas))
    _say("  loss", loss, lo)
    assert abs(loss - lo) <= 1e-5 * max(1.0, abs(lo)) * 10
    gg = unpack(g, grad, h1, h2)
    bound = grad_error_bound(Pd, g, S, betas)
    for k in go:
        err = np.abs(gg[k] - go[k])
        _say(f"  grad {k}: max |err| {err.max():.3e}, max err/bound {np.max(err / (bound[k] + 1e-300)):.3e}")
        assert np.all(err <= bound[k] + 1e-30), k


def test_adam_training_matches_oracle():
    """Adam steps on the GPU against the fp64 oracle, entry by entry.  An
    Adam step moves an entry by lr r with r = m^/(sqrt(v^) + eps), a ratio of
    degree 0 in the gradients (|r| <= 2 over these few steps), so gradients
    known to within relative error rho (grad_error_bound with lam = 6, over
    |g|) move r by at most rho (2 + |r|) <= 4 rho; entries whose gradient may
    change sign within that bound in some step (rho >= 1/4) may move by
    anything Adam allows, at most 3 lr per step.  fp32 storage of the
    parameters adds 2 u |P| per step."""
    n, variant, h1, h2 = 6, "skolem", 48, 40
    g = OM.Geometry(n, variant)
    rng = np.random.default_rng(7)
    P0 = sk.mlp_init(n, variant, h1, h2, seed=9)
    N, B, steps, lr = 45, 16, 4, 1e-3
    S = random_states(g, N, rng)
    betas = rng.uniform(0, 3, size=N)
    P1, last = sk.mlp_train(n, variant, P0, S, betas, steps, B, lr, h1, h2)
    # oracle: the same cyclic minibatches
    Pd = unpack(g, P0, h1, h2)
    M = {k: np.zeros_like(v) for k, v in Pd.items()}
    V = {k: np.zeros_like(v) for k, v in Pd.items()}
    rel = {k: np.zeros_like(v) for k, v in Pd.items()}
    lo = None
    for t in range(steps):
        rows = [(t * B + i) % N for i in range(B)]
        st = [list(S[r]) for r in rows]
        bt = [betas[r] for r in rows]
        bnd = grad_error_bound(Pd, g, st, bt, lam=6.0)
        lo, G = OM.loss_and_grad(Pd, g, st, bt)
        for k in G:
            rel[k] = np.maximum(rel[k], bnd[k] / np.maximum(np.abs(G[k]), 1e-300))
        OM.adam(Pd, G, M, V, t + 1, lr=lr)
    assert abs(last - lo) < 1e-4 * max(1.0, abs(lo))
    got = unpack(g, P1, h1, h2)
    start = unpack(g, P0, h1, h2)
    flipped = 0
    for k in Pd:
        r = rel[k]
        stable = r < 0.25
        tol = np.where(stable, steps * lr * 4 * r, 3 * lr * steps)
        tol = tol + steps * U32 * (np.abs(start[k]) + lr * steps) * 2
        err = np.abs(got[k] - Pd[k])
        flipped += int((~stable).sum())
        _say(f"adam {k}: max |err| {err.max():.3e}, max err/tol {np.max(err / tol):.3e}, "
             f"unstable entries {int((~stable).sum())} of {r.size}")
        assert np.all(err <= tol), k
    # most entries are held to the tight bound
    assert flipped < 0.25 * sum(v.size for v in Pd.values())


def _oracle_decision(Pd, g, a, beta, wp, wa):
    """The oracle's proposal index, margins, log q's and decision."""
    mask = g.valid.reshape(-1)
    z, _ = OM.forward(Pd, OM.features(g, a, beta)[None, :])
    lq = OM.masked_log_softmax(z, mask[None, :])[0]
    q = np.where(mask, np.exp(lq), 0.0)
    cdf = np.cumsum(q)
    u = wp * 2.0 ** -32
    j = int(np.searchsorted(cdf, u * cdf[-1], side="right"))
    j = min(j, g.dout - 1)
    while not mask[j]:
        j -= 1
    margin = min(abs(u * cdf[-1] - cdf[j]), abs(u * cdf[-1] - (cdf[j - 1] if j > 0 else 0.0)))
    return j, margin, lq


@pytest.mark.parametrize("variant,n,h1,h2", [("skolem", 6, 64, 64), ("skolem", 32, 256, 256),
                                            ("hooked", 6, 40, 40)])
def test_mh_step_matches_oracle(variant, n, h1, h2):
    _say("mh step", variant, n)
    g = OM.Geometry(n, variant)
    rng = np.random.default_rng(31 + n)
    B = 200
    P = sk.mlp_init(n, variant, h1, h2, seed=13, scale=2.0)
    Pd = unpack(g, P, h1, h2)
    S = random_states(g, B, rng)
    betas = rng.uniform(0, 3, size=B)
    wp = rng.integers(0, 2 ** 32, size=B, dtype=np.uint64).astype(np.uint32)
    wa = rng.integers(0, 2 ** 32, size=B, dtype=np.uint64).astype(np.uint32)
    r = sk.mlp_mh_step(n, variant, P, S, betas, wp, wa, h1, h2)
    compared = 0
    for i in range(B):
        a = [int(x) for x in S[i]]
        prop = [int(x) for x in r["proposed"][i]]
        diff = [k for k in range(n) if prop[k] != a[k]]
        assert len(diff) <= 1
        jo, margin, lq = _oracle_decision(Pd, g, a, betas[i], int(wp[i]), int(wa[i]))
        if diff:
            k = diff[0]
            jg = k * g.T + prop[k] - 1
        else:  # the proposal re-placed some pair where it already was
            jg = None
        assert all(g.valid[k, prop[k] - 1] for k in range(n))
        if margin > 1e-4:
            if jg is not None:
                assert jg == jo, (i, jg, jo)
            else:
                ko, apo = divmod(jo, g.T)
                assert a[ko] == apo + 1
            assert abs(r["logq_forward"][i] - lq[jo]) < 2e-4 * max(1.0, abs(lq[jo]))
            ko, apo = divmod(jo, g.T)
            b = list(a)
            old = b[ko]
            b[ko] = apo + 1
            zb, _ = OM.forward(Pd, OM.features(g, b, betas[i])[None, :])
            lqb = OM.masked_log_softmax(zb, g.valid.reshape(-1)[None, :])[0]
            lrev = lqb[ko * g.T + old - 1]
            assert abs(r["logq_reverse"][i] - lrev) < 2e-4 * max(1.0, abs(lrev))
            log_alpha = -betas[i] * (g.energy(b) - g.energy(a)) + lrev - lq[jo]
            u = int(wa[i]) * 2.0 ** -32
            if u > 0 and abs(math.log(u) - min(0.0, log_alpha)) > 1e-3:
                acc = math.log(u) < min(0.0, log_alpha)
                assert bool(r["accepted"][i]) == acc, i
                assert [int(x) for x in r["states"][i]] == (b if acc else a)
                compared += 1
    _say("  decisions compared:", compared, "of", B)
    assert compared > 0.9 * B


def _boltzmann_table(g: OM.Geometry, beta: float):
    """All configurations of a small instance, their energies and exact law."""
    choices = [list(np.nonzero(g.valid[k])[0] + 1) for k in range(g.n)]
    confs = np.array(list(itertools.product(*choices)), dtype=np.uint8)
    E = np.array([g.energy(list(c)) for c in confs])
    w = np.exp(-beta * (E - E.min()))
    return confs, E, w / w.sum()


@pytest.mark.parametrize("beta", [0.0, 1.0, 2.5])
def test_mh_step_keeps_boltzmann_law(beta):
    """Start from exact samples of exp(-beta E) and apply learned moves with a
    deliberately skewed (random, large-weight) network: the law of the energy
    must not move.  A missing or inverted Hastings factor skews it."""
    n, variant, h1, h2 = 4, "skolem", 32, 32
    g = OM.Geometry(n, variant)
    confs, E, p = _boltzmann_table(g, beta)
    rng = np.random.default_rng(1000 + int(10 * beta))
    B, steps = 20000, 6
    S = confs[rng.choice(len(confs), size=B, p=p)]
    P = sk.mlp_init(n, variant, h1, h2, seed=77, scale=4.0)
    betas = np.full(B, beta)
    acc = 0
    for _ in range(steps):
        wp = rng.integers(0, 2 ** 32, size=B, dtype=np.uint64).astype(np.uint32)
        wa = rng.integers(0, 2 ** 32, size=B, dtype=np.uint64).astype(np.uint32)
        r = sk.mlp_mh_step(n, variant, P, S, betas, wp, wa, h1, h2)
        S = r["states"]
        acc += int(r["accepted"].sum())
    Ef = np.array([g.energy(list(s)) for s in S])
    Hmax = E.max() + 1
    expect = np.array([p[E == e].sum() for e in range(Hmax)]) * B
    got = np.bincount(Ef, minlength=Hmax)[:Hmax]
    keep = expect > 5
    chi2 = float(((got[keep] - expect[keep]) ** 2 / expect[keep]).sum())
    dof = int(keep.sum()) - 1
    _say("beta", beta, "acceptance", acc / (B * steps), "chi2", chi2, "dof", dof, got, np.round(expect))
    assert acc > 0.05 * B * steps
    # chi-square with dof <= 8: P(chi2 > 30) < 3e-4
    assert chi2 < 30


def test_invalid_inputs():
    P = sk.mlp_init(4, "skolem", 8, 8)
    with pytest.raises(sk.SkolemError):
        sk.mlp_forward(4, "skolem", P, np.array([[1, 1, 1, 9]], dtype=np.uint8), [0.5], 8, 8)  # 9 + 4 > 8
    with pytest.raises(sk.SkolemError):
        sk.mlp_forward(4, "skolem", P, np.array([[0, 1, 1, 1]], dtype=np.uint8), [0.5], 8, 8)  # position 0
