"""Pins for the oracle of the learned importance proposal: analytic
gradients against finite differences, Adam's first step in closed form,
bfloat16 rounding on ties, the quantisation's guarantees, the features
against a direct scan of the edge list, and the importance-sampling
estimator against its exact expectation and variance from enumeration."""
import math
from fractions import Fraction

import numpy as np
import pytest

import oracle
import synthgraph as sg
from oracle import learn

M40 = sg.motif_bytes(sg.MOTIFS["M4-0"])
SIX = [sg.motif_bytes(sg.MOTIFS[n]) for n in sg.SIX_MOTIFS]


def rand_params(rng, scale=0.3):
    return (rng.standard_normal(learn.N_PARAMS) * scale).astype(np.float32)


# ------------------------------------------------------------------ MLP ----
def test_param_count():
    assert learn.N_PARAMS == 8 * 64 + 64 + 64 * 64 + 64 + 64 + 1 == 4801


def test_gradient_matches_finite_differences():
    rng = np.random.default_rng(3)
    P = rand_params(rng).astype(np.float64)
    F = rng.standard_normal((40, 8))
    y = (rng.random(40) < 0.4).astype(np.float64)
    loss, G = learn.grad(P, F, y, bf16=False)

    def L(p):
        # the same function in binary64 throughout (no float32 parameter cast)
        W1 = p[learn.OFF_W1:learn.OFF_B1].reshape(64, 8)
        b1 = p[learn.OFF_B1:learn.OFF_W2]
        W2 = p[learn.OFF_W2:learn.OFF_B2].reshape(64, 64)
        b2 = p[learn.OFF_B2:learn.OFF_W3]
        w3 = p[learn.OFF_W3:learn.OFF_B3]
        b3 = p[learn.OFF_B3]
        h1 = np.maximum(F @ W1.T + b1, 0)
        h2 = np.maximum(h1 @ W2.T + b2, 0)
        z3 = h2 @ w3 + b3
        return float(np.mean(y * np.logaddexp(0, -z3) + (1 - y) * np.logaddexp(0, z3)))

    # the float32 cast inside learn.grad must not matter for these parameters
    P = P.astype(np.float32).astype(np.float64)
    loss, G = learn.grad(P, F, y, bf16=False)
    assert abs(loss - L(P)) < 1e-12
    idx = np.concatenate([rng.choice(np.arange(learn.OFF_W1, learn.OFF_B1), 10, replace=False),
                          rng.choice(np.arange(learn.OFF_B1, learn.OFF_W2), 5, replace=False),
                          rng.choice(np.arange(learn.OFF_W2, learn.OFF_B2), 20, replace=False),
                          rng.choice(np.arange(learn.OFF_B2, learn.OFF_W3), 5, replace=False),
                          rng.choice(np.arange(learn.OFF_W3, learn.OFF_B3), 8, replace=False),
                          [learn.OFF_B3]])
    h = 1e-6
    for i in idx:
        e = np.zeros_like(P)
        e[i] = h
        fd = (L(P + e) - L(P - e)) / (2 * h)
        assert abs(fd - G[i]) <= 1e-6 * max(1.0, abs(fd)) + 1e-9, (i, fd, G[i])


def test_bf16_rounding_ties_and_values():
    v = np.array([1.0, 1 + 2**-8, 1 + 3 * 2**-8, -2.5, 3.0e38, 1 + 2**-7], np.float32)
    r = learn.bf16_round(v)
    assert r[0] == 1.0
    assert r[1] == 1.0                 # tie -> even
    assert r[2] == 1 + 2**-6           # tie -> even (upwards)
    assert r[3] == -2.5
    assert r[5] == 1 + 2**-7           # representable
    assert np.all(learn.bf16_from_bits(learn.bf16_bits(v)) == r)


def test_adam_first_step_closed_form():
    """At step 1 the bias-corrected moments are g and g^2, so the update is
    lr * g / (|g| + eps)."""
    rng = np.random.default_rng(1)
    p = rng.standard_normal(50)
    g = rng.standard_normal(50)
    lr, eps = 1e-3, 1e-8
    p1, m, v = learn.adam_step(p, np.zeros(50), np.zeros(50), g, 1, lr, eps=eps)
    assert np.allclose(p1, p - lr * g / (np.abs(g) + eps), rtol=0, atol=1e-15)
    assert np.allclose(m, 0.1 * g) and np.allclose(v, 0.001 * g * g)


def test_forward_bf16_close_to_exact():
    rng = np.random.default_rng(4)
    P = rand_params(rng)
    F = rng.standard_normal((200, 8))
    a = learn.forward(P, F, bf16=True)["g"]
    b = learn.forward(P, F, bf16=False)["g"]
    assert np.max(np.abs(a - b)) < 0.05


def _torch_forward(P, F):
    """The same network through torch.nn.functional in float64 on the CPU: a
    library implementation of linear, ReLU and sigmoid, independent of the
    oracle's numpy code.  torch's linear takes weights as [out, in], which is
    the row = unit layout of the parameter vector."""
    import torch
    import torch.nn.functional as tF
    p = torch.from_numpy(np.asarray(P, np.float64))
    x = torch.from_numpy(np.asarray(F, np.float64))
    W1 = p[learn.OFF_W1:learn.OFF_B1].reshape(64, 8)
    W2 = p[learn.OFF_W2:learn.OFF_B2].reshape(64, 64)
    w3 = p[learn.OFF_W3:learn.OFF_B3].reshape(1, 64)
    h1 = tF.relu(tF.linear(x, W1, p[learn.OFF_B1:learn.OFF_W2]))
    h2 = tF.relu(tF.linear(h1, W2, p[learn.OFF_B2:learn.OFF_W3]))
    z3 = tF.linear(h2, w3, p[learn.OFF_B3:learn.OFF_B3 + 1])[:, 0]
    return z3, torch.sigmoid(z3)


def test_forward_and_loss_match_torch_float64():
    import torch
    import torch.nn.functional as tF
    rng = np.random.default_rng(8)
    P = rand_params(rng, scale=0.4)
    F = rng.standard_normal((300, 8)) * 2.0
    y = (rng.random(300) < 0.3).astype(np.float64)
    c = learn.forward(P, F, bf16=False)
    z3, g = _torch_forward(P, F)
    assert np.allclose(c["z3"], z3.numpy(), rtol=1e-12, atol=1e-12)
    assert np.allclose(c["g"], g.numpy(), rtol=1e-12, atol=1e-14)
    ref = tF.binary_cross_entropy_with_logits(z3, torch.from_numpy(y)).item()
    assert abs(learn.bce_loss(c["z3"], y) - ref) <= 1e-12 * max(1.0, abs(ref))


def test_gradient_matches_torch_autograd_float64():
    import torch
    import torch.nn.functional as tF
    rng = np.random.default_rng(9)
    P = rand_params(rng, scale=0.4).astype(np.float64)
    F = rng.standard_normal((64, 8))
    y = (rng.random(64) < 0.5).astype(np.float64)
    loss, G = learn.grad(P, F, y, bf16=False)
    p = torch.from_numpy(P.copy()).requires_grad_(True)
    x = torch.from_numpy(F)
    h1 = tF.relu(tF.linear(x, p[learn.OFF_W1:learn.OFF_B1].reshape(64, 8),
                           p[learn.OFF_B1:learn.OFF_W2]))
    h2 = tF.relu(tF.linear(h1, p[learn.OFF_W2:learn.OFF_B2].reshape(64, 64),
                           p[learn.OFF_B2:learn.OFF_W3]))
    z3 = (h2 @ p[learn.OFF_W3:learn.OFF_B3]) + p[learn.OFF_B3]
    L = tF.binary_cross_entropy_with_logits(z3, torch.from_numpy(y))
    L.backward()
    assert abs(loss - L.item()) <= 1e-12
    assert np.allclose(G, p.grad.numpy(), rtol=1e-10, atol=1e-13)


def _zero_params():
    return np.zeros(learn.N_PARAMS, np.float32)


def test_forward_hand_computed_constant_second_layer():
    """W2 = 0 makes the output independent of the input:
    g = sigmoid(sum_i w3_i relu(b2_i) + b3).  With b2 = (1, -1, 2, 0, ...),
    w3 = (0.5, 3, 0.25, 7, ...) and b3 = -1 this is sigmoid(0.5 + 0.5 - 1) =
    1/2; a missing second ReLU would add -3, a wrong output bias would move
    it off 0."""
    P = _zero_params()
    P[learn.OFF_B2:learn.OFF_B2 + 4] = [1.0, -1.0, 2.0, 0.0]
    P[learn.OFF_W3:learn.OFF_W3 + 4] = [0.5, 3.0, 0.25, 7.0]
    P[learn.OFF_B3] = -1.0
    P[learn.OFF_W1:learn.OFF_B1] = np.linspace(-1, 1, 512, dtype=np.float32)  # irrelevant
    F = np.random.default_rng(0).standard_normal((5, 8))
    for bf16 in (False, True):
        c = learn.forward(P, F, bf16=bf16)
        assert np.all(c["z3"] == 0.0) and np.all(c["g"] == 0.5)
    # loss at z3 = 0 is ln 2 whatever the labels
    assert abs(learn.bce_loss(np.zeros(4), [0, 1, 1, 0]) - math.log(2.0)) < 1e-15


def test_forward_hand_computed_single_path():
    """One live unit in each layer: unit 0 of layer 1 reads feature 2 only
    (W1[0][2] = 2, row = unit), b1[0] = -1; unit 0 of layer 2 is
    -h1_0 + 1; the output is that unit.  For f_2 = 3: z1 = 5, z2 = -4 ->
    relu 0, g = sigmoid(b3) = sigmoid(0.25).  For f_2 = 0.2: z1 = -0.6 ->
    relu 0, z2 = 1, g = sigmoid(1.25).  A transposed W1 (unit 2 reading
    feature 0), a missing first ReLU (z2 = 1.6) or a missing second ReLU
    (z2 = -4 kept) each change one of the two values."""
    P = _zero_params()
    P[learn.OFF_W1 + 0 * 8 + 2] = 2.0
    P[learn.OFF_B1 + 0] = -1.0
    P[learn.OFF_W2 + 0 * 64 + 0] = -1.0
    P[learn.OFF_B2 + 0] = 1.0
    P[learn.OFF_W3 + 0] = 1.0
    P[learn.OFF_B3] = 0.25
    F = np.zeros((3, 8))
    F[0, 2] = 3.0
    F[1, 2] = 0.2
    F[2, 0] = 5.0        # feature 0 only: unit 0 sees nothing
    c = learn.forward(P, F, bf16=False)
    sig = lambda z: 1.0 / (1.0 + math.exp(-z))
    assert np.allclose(c["z3"], [0.25, 1.25, 1.25], rtol=0, atol=1e-15)
    assert np.allclose(c["g"], [sig(0.25), sig(1.25), sig(1.25)], rtol=0, atol=1e-15)
    # every value here is exact in bfloat16
    assert np.allclose(learn.forward(P, F, bf16=True)["z3"], [0.25, 1.25, 1.25], atol=0)
    # loss against labels (1, 0, 1): -log g, -log(1 - g), -log g, averaged
    y = np.array([1.0, 0.0, 1.0])
    want = (-math.log(sig(0.25)) - math.log(1 - sig(1.25)) - math.log(sig(1.25))) / 3
    assert abs(learn.bce_loss(c["z3"], y) - want) < 1e-15


# --------------------------------------------------------- quantisation ----
def test_quant_shift():
    assert learn.quant_shift(0) == 16
    assert learn.quant_shift(1) == 16
    assert learn.quant_shift(2**46) == 16          # bitlen 47 -> 16
    assert learn.quant_shift(2**50) == 12          # bitlen 51
    assert learn.quant_shift(2**62) == 1           # bitlen 63 -> clamp
    assert learn.quant_shift(2**64 - 1) == 1


def test_quantize_range_monotone_and_bound():
    rng = np.random.default_rng(2)
    g = np.sort(rng.random(5000).astype(np.float32))
    g[0], g[-1] = 0.0, 1.0
    for W in (5, 2**40, 2**50, 2**61):
        s = learn.quant_shift(W)
        h = learn.quantize(g, W, 0.1)
        assert h.min() >= 1 and h.max() == 2**s
        assert np.all(np.diff(h.astype(np.int64)) >= 0)
        assert h[0] == max(1, math.floor(float(np.float32(0.1) * np.float32(2.0**s)) + 0.5))
        # the proposal total never overflows: W * 2^s < 2^63 for bitlen(W) <= 62
        if W.bit_length() <= 62:
            assert W * int(h.max()) < 2**63
    # normalised: the largest score maps to 2^s, order is kept
    gs = (g * np.float32(0.02)).astype(np.float32)
    hn = learn.quantize(gs, 2**40, 0.05, normalize=True)
    assert hn.max() == 2**16 and np.all(np.diff(hn.astype(np.int64)) >= 0)
    assert hn[0] == math.floor(float(np.float32(0.05) * np.float32(2.0**16)) + 0.5)
    h = learn.quantize(np.array([np.nan, -1.0, 2.0], np.float32), 1000, 0.1)
    assert list(h) == [learn.quantize(np.float32([0.0]), 1000)[0], h[0], 2**16]


# ------------------------------------------------------------- features ----
def test_features_by_direct_scan():
    for seed in range(3):
        g = sg.gen_micro(seed + 30, n=6, m=40, t_span=25)
        og = oracle.OracleGraph.from_graph(g)
        for delta in (0, 4, 11):
            w = og.weights(delta)
            F = og.features(w)
            out = og.orders()["out_eid"]
            for p in range(g.m):
                e = out[p]
                u, v, t = int(g.src[e]), int(g.dst[e]), int(g.t[e])
                ins = [int(g.t[i]) for i in range(g.m) if g.dst[i] == u and t - delta <= g.t[i] <= t]
                outs = [int(g.t[i]) for i in range(g.m) if g.src[i] == v and t <= g.t[i] <= t + delta]
                a, b = len(ins), len(outs)
                want = [math.log1p(a), math.log1p(b), math.log1p(a * b),
                        (t - min(ins)) / delta if a and delta else 0.0,
                        (max(outs) - t) / delta if b and delta else 0.0,
                        math.log1p(sum(1 for i in range(g.m) if g.src[i] == u and g.dst[i] == v
                                       and abs(int(g.t[i]) - t) <= delta)),
                        math.log1p(sum(1 for i in range(g.m) if g.src[i] == v and g.dst[i] == u
                                       and abs(int(g.t[i]) - t) <= delta)),
                        0.5 * math.log1p(
                            (np.mean([min(int(np.sum(g.dst == g.src[i])), 65535) ** 2
                                      for i in range(g.m)
                                      if g.dst[i] == u and t - delta <= g.t[i] <= t])
                             if a else 0.0) *
                            (np.mean([min(int(np.sum(g.src == g.dst[i])), 65535) ** 2
                                      for i in range(g.m)
                                      if g.src[i] == v and t <= g.t[i] <= t + delta])
                             if b else 0.0))]
                assert np.allclose(F[p], want, rtol=1e-15, atol=0), (seed, delta, p)


# ------------------------------------------------- importance sampling ----
def _paths_exact(og, w, hw, motif):
    """Exact C, E_q[X/h * Q] pieces and Var of plain and IS from enumeration."""
    orders = og.orders()
    ie, oe = orders["in_eid"], orders["out_eid"]
    W, Q = w.W, hw.W
    C = 0
    s_plain = Fraction(0)
    s_is = Fraction(0)
    for p in range(og.m):
        hp = int(hw.h[p])
        for j1 in range(int(w.a[p])):
            for j3 in range(int(w.b[p])):
                _, X = og.check_motif(motif, w.delta, int(ie[w.lo_in[p] + j1]), int(oe[p]),
                                      int(oe[w.lo_out[p] + j3]))
                C += X
                s_plain += X * X
                s_is += Fraction(X * X, hp)
    var_plain = s_plain * W - C * C    # E_w[(X W)^2] - C^2
    var_is = s_is * Q - C * C          # E_q[(X Q / h)^2] - C^2
    return C, var_plain, var_is


@pytest.mark.parametrize("seed", range(4))
def test_is_exact_expectation_equals_count(seed):
    M = sg.MOTIFS[sg.SIX_MOTIFS[seed % 6]]
    g = sg.gen_micro_planted(seed, M, copies=3, n=7, noise=10)
    og = oracle.OracleGraph.from_graph(g)
    mb = sg.motif_bytes(M)
    rng = np.random.default_rng(seed)
    for delta in (4, 9, 40):
        w = og.weights(delta)
        s = learn.quant_shift(w.W)
        # arbitrary h: expectation within the 2^-64 truncation of the count
        h = rng.integers(1, 2**s + 1, size=og.m).astype(np.uint32)
        hw = og.proposal(w, h)
        E, C = learn.is_expectation(og, w, hw, mb)
        assert C == og.brute_count(mb, delta)
        n_paths = int(np.sum(w.a.astype(np.int64) * w.b.astype(np.int64)))
        assert abs(E - C) <= Fraction(n_paths * 2**s, 2**64)
        # powers of two: the correction is exact
        h2 = (1 << rng.integers(0, s + 1, size=og.m)).astype(np.uint32)
        E2, C2 = learn.is_expectation(og, w, og.proposal(w, h2), mb)
        assert E2 == C2 == C


def test_is_with_constant_h_reduces_to_plain_bit_exactly():
    g = sg.gen_tiny()
    og = oracle.OracleGraph.from_graph(g)
    for delta in (3600, 20000):
        w = og.weights(delta)
        s = learn.quant_shift(w.W)
        hw = og.proposal(w, np.full(og.m, 2**s, np.uint32))
        assert hw.W == w.W << s
        P = og.sample(w, SIX, 20000, 5, per_sample=True)
        I = og.sample(hw, SIX, 20000, 5, per_sample=True)
        assert P.status == I.status == 0
        assert np.array_equal(P.e2, I.e2) and np.array_equal(P.X, I.X)
        assert I.cnt == [c << (64 - s) for c in P.cnt]
        assert np.array_equal(P.est.view(np.uint64), I.est.view(np.uint64))
        assert np.array_equal(P.P, I.P)


def test_is_unbiased_over_seeds_with_exact_variance():
    """z-test of the IS estimate over independent seeds, with the exact
    variance from enumeration; also the variance reduction of a proposal
    that favours edges whose paths close."""
    g = sg.gen_micro_planted(2, sg.MOTIFS["M4-0"], copies=4, n=8, noise=14)
    og = oracle.OracleGraph.from_graph(g)
    w = og.weights(12)
    s = learn.quant_shift(w.W)
    # ideal-ish proposal: 2^s where some path through p closes, else 1
    orders = og.orders()
    ie, oe = orders["in_eid"], orders["out_eid"]
    h = np.ones(og.m, np.uint32)
    for p in range(og.m):
        for j1 in range(int(w.a[p])):
            for j3 in range(int(w.b[p])):
                if og.check_motif(M40, 12, int(ie[w.lo_in[p] + j1]), int(oe[p]),
                                  int(oe[w.lo_out[p] + j3]))[1]:
                    h[p] = 2**s
    hw = og.proposal(w, h)
    C, var_plain, var_is = _paths_exact(og, w, hw, M40)
    assert C > 0 and var_is < var_plain
    k, R = 4000, 40
    ests = np.array([og.sample(hw, [M40], k, seed).est[0] for seed in range(1, R + 1)])
    z = (ests.mean() - C) / math.sqrt(float(var_is) / k / R)
    assert abs(z) < 4.5, z
    # the sample second moment estimates E[(X/h)^2]
    e = og.sample(hw, [M40], 200000, 77)
    m2_exact = (var_is + C * C) / (hw.W * hw.W)
    assert abs(e.m2[0] / 200000 - float(m2_exact)) < 0.05 * float(m2_exact)
