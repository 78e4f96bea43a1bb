"""GPU parity of the learned importance proposal through the C ABI:
features against the oracle's binary64 features, the MFMA network (forward
and gradients) against the oracle's binary64 network on the same bfloat16
inputs, Adam, the float32 quantisation (bit-exact), the proposal scan and
the importance-sampling estimator (bit-exact on all integer work and the
estimate), and the gain of a trained proposal over the method."""
import math

import numpy as np
import pytest

import synthgraph as sg
from test_gpu_parity import _u64, build_both

pytestmark = pytest.mark.gpu

SIX = [sg.MOTIFS[n] for n in sg.SIX_MOTIFS]
M40 = sg.MOTIFS["M4-0"]


@pytest.fixture(scope="module")
def tcb():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2409_08975_amd as tcb
    tcb.lib()
    return tcb


@pytest.fixture(scope="module")
def torch_mod():
    import torch
    return torch


@pytest.fixture(scope="module")
def tiny(tcb, torch_mod):
    g = sg.gen_tiny()
    G, og = build_both(tcb, torch_mod, g)
    return g, G, og


def _bf16_to_f64(bits):
    u = np.asarray(bits).astype(np.uint16).astype(np.uint32) << 16
    return u.view(np.float32).astype(np.float64)


# ------------------------------------------------------------- features ----
@pytest.mark.parametrize("delta", [0, 3600, 20000])
def test_features_match_oracle(tcb, tiny, delta):
    g, G, og = tiny
    Wt = tcb.tc_path_weights(G, delta)
    F = tcb.tc_edge_features(G, Wt).cpu().numpy()
    got = _bf16_to_f64(F.view(np.uint16))
    want = og.features(og.weights(delta))
    # float32 evaluation then bfloat16 rounding: within 2^-8 relative
    assert np.all(np.abs(got - want) <= 2.0**-8 * np.abs(want) + 1e-6), \
        np.max(np.abs(got - want) / (np.abs(want) + 1e-6))


def test_features_planted_micro(tcb, torch_mod):
    g = sg.gen_micro_planted(1, M40, copies=3, n=7, noise=12)
    G, og = build_both(tcb, torch_mod, g)
    for delta in (3, 9, 40):
        F = tcb.tc_edge_features(G, tcb.tc_path_weights(G, delta)).cpu().numpy()
        got = _bf16_to_f64(F.view(np.uint16))
        want = og.features(og.weights(delta))
        assert np.all(np.abs(got - want) <= 2.0**-8 * np.abs(want) + 1e-6)


# -------------------------------------------------------------- network ----
def _net_inputs(torch, n, seed):
    P = sg.random_params(seed)
    Fb = sg.random_bf16_bits(seed + 1, (n, 8))
    return P, Fb, torch.from_numpy(P).cuda(), torch.from_numpy(Fb.view(np.int16)).cuda()


@pytest.mark.parametrize("n", [1, 31, 32, 1000, 4133])
def test_mlp_forward_matches_oracle(tcb, torch_mod, n):
    from oracle import learn
    P, Fb, Pd, Fd = _net_inputs(torch_mod, n, 7 + n)
    g = tcb.tc_mlp_forward(Pd, Fd).cpu().numpy().astype(np.float64)
    want = learn.forward(P, _bf16_to_f64(Fb), bf16=True)["g"]
    err = np.abs(g - want)
    assert err.max() <= 4e-3 and err.mean() <= 4e-4, (err.max(), err.mean())


@pytest.mark.parametrize("n,with_rows,cap", [(64, False, 0.0), (1000, True, 0.0),
                                             (20011, True, 0.0), (5000, True, 3.0)])
def test_mlp_grad_matches_oracle(tcb, torch_mod, n, with_rows, cap):
    from oracle import learn
    torch = torch_mod
    P, Fb, Pd, Fd = _net_inputs(torch, 3000, 100 + n)
    rng = np.random.default_rng(n)
    rows = rng.integers(0, 3000, size=n).astype(np.uint32) if with_rows else np.arange(n, dtype=np.uint32)
    X = sg.random_counts(200 + n, n)
    grad, loss = tcb.tc_mlp_grad(Pd, Fd, torch.from_numpy(rows.view(np.int32)).cuda() if with_rows else None,
                                 torch.from_numpy(X.view(np.int64)).cuda(), label_cap=cap)
    grad = grad.cpu().numpy().astype(np.float64)
    y = ((X > 0).astype(np.float64) if cap == 0 else
         np.minimum(np.float32(1), X.astype(np.float32) / np.float32(cap)).astype(np.float64))
    lw, gw = learn.grad(P, _bf16_to_f64(Fb)[rows], y, bf16=True)
    assert abs(float(loss.item()) - lw) <= 1e-4 * abs(lw) + 1e-6
    blocks = [(learn.OFF_W1, learn.OFF_B1), (learn.OFF_B1, learn.OFF_W2),
              (learn.OFF_W2, learn.OFF_B2), (learn.OFF_B2, learn.OFF_W3),
              (learn.OFF_W3, learn.OFF_B3), (learn.OFF_B3, learn.N_PARAMS)]
    for a, b in blocks:
        rel = np.linalg.norm(grad[a:b] - gw[a:b]) / max(np.linalg.norm(gw[a:b]), 1e-12)
        assert rel <= 1e-2, (a, b, rel)


def test_mlp_grad_deterministic(tcb, torch_mod):
    torch = torch_mod
    P, Fb, Pd, Fd = _net_inputs(torch, 50000, 5)
    X = torch.from_numpy(sg.random_counts(9, 50000).view(np.int64)).cuda()
    g1, l1 = tcb.tc_mlp_grad(Pd, Fd, None, X)
    g2, l2 = tcb.tc_mlp_grad(Pd, Fd, None, X)
    assert torch.equal(g1, g2) and torch.equal(l1, l2)


def test_adam_matches_oracle(tcb, torch_mod):
    from oracle import learn
    torch = torch_mod
    rng = np.random.default_rng(3)
    p = rng.standard_normal(learn.N_PARAMS).astype(np.float32)
    m = (rng.standard_normal(learn.N_PARAMS) * 0.01).astype(np.float32)
    v = (rng.random(learn.N_PARAMS) * 1e-3).astype(np.float32)
    gr = rng.standard_normal(learn.N_PARAMS).astype(np.float32)
    pd, od = torch.from_numpy(p.copy()).cuda(), torch.from_numpy(np.concatenate([m, v])).cuda()
    tcb.tc_mlp_adam(pd, od, torch.from_numpy(gr).cuda(), 3, 1e-3)
    wp, wm, wv = learn.adam_step(p, m, v, gr.astype(np.float64), 3, 1e-3)
    # float32 arithmetic: a few ulps of the largest term (|g| < 5, m ~ 0.1 g,
    # v ~ 1e-3 g^2), so absolute bounds near cancellation
    assert np.allclose(pd.cpu().numpy(), wp, rtol=1e-5, atol=1e-7)
    assert np.allclose(od[:learn.N_PARAMS].cpu().numpy(), wm, rtol=1e-5, atol=2e-7)
    assert np.allclose(od[learn.N_PARAMS:].cpu().numpy(), wv, rtol=1e-5, atol=1e-9)


# --------------------------------------------------------- quantisation ----
def test_quantize_bit_exact(tcb, tiny, torch_mod):
    from oracle import learn
    torch = torch_mod
    g, G, og = tiny
    for delta in (3600, 86400):
        Wt = tcb.tc_path_weights(G, delta)
        rng = np.random.default_rng(delta)
        gv = rng.random(G.m).astype(np.float32)
        gv[:5] = [0.0, 1.0, np.nan, -0.5, 2.0]
        h = tcb.tc_quantize_proposal(Wt, torch.from_numpy(gv).cuda(), 0.1).cpu().numpy()
        want = learn.quantize(gv, Wt.total(), 0.1)
        assert np.array_equal(h.view(np.uint32), want)
        # normalised by the maximum score
        gs = (gv * np.float32(0.03)).astype(np.float32)
        hn = tcb.tc_quantize_proposal(Wt, torch.from_numpy(gs).cuda(), 0.05,
                                      normalize=True).cpu().numpy()
        assert np.array_equal(hn.view(np.uint32), learn.quantize(gs, Wt.total(), 0.05, True))


# ------------------------------------------------ importance sampling ----
def _seeded_h(og, w, seed):
    from oracle import learn
    s = learn.quant_shift(w.W)
    rng = np.random.default_rng(seed)
    return rng.integers(1, 2**s + 1, size=og.m).astype(np.uint32)


def _is_pair(tcb, torch, G, og, delta, seed):
    Wt = tcb.tc_path_weights(G, delta)
    ow = og.weights(delta)
    h = _seeded_h(og, ow, seed)
    Wq = tcb.tc_proposal_weights(G, Wt, torch.from_numpy(h.view(np.int32)).cuda())
    return Wt, ow, Wq, og.proposal(ow, h)


@pytest.mark.parametrize("delta", [3600, 20000, 86400])
def test_proposal_scan_bit_exact(tcb, tiny, torch_mod, delta):
    g, G, og = tiny
    Wt, ow, Wq, oq = _is_pair(tcb, torch_mod, G, og, delta, delta)
    assert np.array_equal(_u64(Wq.view("S", torch_mod.int64, G.m + 1)), oq.S)
    assert Wq.status() == oq.status == 0


@pytest.mark.parametrize("delta,seed,stream", [(3600, 1, 0), (20000, 9, 3), (86400, 2**33 + 1, 7)])
def test_is_sampler_bit_exact(tcb, tiny, torch_mod, delta, seed, stream):
    g, G, og = tiny
    Wt, ow, Wq, oq = _is_pair(tcb, torch_mod, G, og, delta, seed)
    k = 50000
    R = tcb.tc_sample_estimate(G, Wq, SIX, k, seed, stream, 0, per_sample=True, moments=True)
    E = og.sample(oq, [sg.motif_bytes(M) for M in SIX], k, seed, stream, per_sample=True)
    assert (int(R.status.item()) & 0xFFFFFFFF) == E.status == 0
    assert np.array_equal(R.e1.cpu().numpy(), E.e1) and np.array_equal(R.e3.cpu().numpy(), E.e3)
    assert np.array_equal(R.P.cpu().numpy().view(np.uint32), E.P)
    assert np.array_equal(_u64(R.X), E.X)
    assert R.counts() == E.cnt
    assert np.array_equal(_u64(R.hits), E.hits)
    assert np.array_equal(R.estimate.cpu().numpy().view(np.uint64), E.est.view(np.uint64))
    m2 = R.m2.cpu().numpy()
    assert np.allclose(m2, E.m2, rtol=1e-12, atol=0)


def test_is_constant_h_equals_method(tcb, tiny, torch_mod):
    """h = 2^s everywhere: the importance-sampling estimate is the method's
    estimate bit for bit (same samples, exact correction)."""
    from oracle import learn
    torch = torch_mod
    g, G, og = tiny
    Wt = tcb.tc_path_weights(G, 20000)
    s = learn.quant_shift(Wt.total())
    h = torch.full((G.m,), 2**s, dtype=torch.int32, device="cuda")
    Wq = tcb.tc_proposal_weights(G, Wt, h)
    a = tcb.tc_sample_estimate(G, Wt, SIX, 40000, 3, per_sample=True)
    b = tcb.tc_sample_estimate(G, Wq, SIX, 40000, 3, per_sample=True)
    assert np.array_equal(_u64(a.X), _u64(b.X))
    assert b.counts() == [c << (64 - s) for c in a.counts()]
    assert np.array_equal(a.estimate.cpu().numpy().view(np.uint64),
                          b.estimate.cpu().numpy().view(np.uint64))


def test_is_in_batch_with_method_weights(tcb, tiny, torch_mod):
    g, G, og = tiny
    Wt, ow, Wq, oq = _is_pair(tcb, torch_mod, G, og, 20000, 4)
    W2 = tcb.tc_path_weights(G, 3600)
    outs = tcb.tc_batch_estimate(G, [Wt, Wq, W2], SIX, 30000, 6, per_sample=True)
    for o, w in zip(outs, [Wt, Wq, W2]):
        r = tcb.tc_sample_estimate(G, w, SIX, 30000, 6, per_sample=True)
        assert o.counts() == r.counts()
        assert np.array_equal(_u64(o.X), _u64(r.X))
        assert np.array_equal(o.estimate.cpu().numpy().view(np.uint64),
                              r.estimate.cpu().numpy().view(np.uint64))


# ------------------------------------------------------------ the gain ----
def test_trained_proposal_reduces_variance(tcb, torch_mod):
    """Train on 2*10^5 closure labels of the medium-shaped graph (smaller
    vertex and edge counts, same recipe), then compare the per-sample
    variance of the importance-sampling estimator with the method's on
    independent streams.  The proposal must lower the variance, and both
    estimates must agree within their standard errors."""
    from paper_2409_08975_amd import learned
    torch = torch_mod
    g = sg.gen_medium(seed=1002, n=100000, m=2000000)
    G = tcb.tc_build_graph(g.n, *[torch.from_numpy(a).cuda() for a in (g.src, g.dst, g.t)])
    Wt = tcb.tc_path_weights(G, 86400)
    lp = learned.LearnedProposal(G, Wt, M40, seed=11)
    losses = lp.fit(n_labels=200000, epochs=4, batch=4096, lr=3e-3).cpu().numpy()
    assert np.all(np.isfinite(losses)) and losses[-1] < losses[0]
    lp.build_proposal()
    assert lp.proposal.status() == 0
    mp, mi = lp.pilot(2 * 10**6, 12345)
    print(f"variance ratio (method / learned) = {mp.var / mi.var:.3f}; "
          f"estimates {mp.estimate:.6g} +- {mp.stderr:.3g} and {mi.estimate:.6g} +- {mi.stderr:.3g}")
    assert mi.var < mp.var
    z = (mp.estimate - mi.estimate) / math.sqrt(mp.stderr ** 2 + mi.stderr ** 2)
    assert abs(z) < 5.0


@pytest.fixture(scope="module")
def medium_graph(tcb, torch_mod):
    """The learned-proposal workload: the medium graph (10^6 vertices,
    2*10^7 edges), delta = 86,400."""
    torch = torch_mod
    g = sg.gen_medium()
    G = tcb.tc_build_graph(g.n, *[torch.from_numpy(a).cuda() for a in (g.src, g.dst, g.t)],
                           check=True)
    Wt = tcb.tc_path_weights(G, 86400)
    return G, Wt


@pytest.mark.parametrize("variant", ["configured", "tuned"])
def test_learned_proposal_on_medium_graph(tcb, medium_graph, variant):
    """On the medium graph with 10^6 training labels: the configured
    proposal (eps = 0.1, labels y = [X > 0]) and the tuned one (eps = 0.01,
    soft labels, normalised scores).  Each estimate agrees with the method's
    within their standard errors (unbiasedness), and each lowers the
    per-sample variance (measured ratios 1.034 for the configured proposal,
    1.346 for the tuned one; asserted: above 1.0 and above 1.2 -- the runs
    are deterministic, the margins allow for changes of launch shape)."""
    from paper_2409_08975_amd import learned
    G, Wt = medium_graph
    if variant == "configured":
        lp = learned.LearnedProposal(G, Wt, M40, eps=0.1, seed=11, normalize=False)
        losses = lp.fit(n_labels=10**6, epochs=8, batch=8192, lr=3e-3, label_cap=0.0)
        margin = 1.0
    else:
        lp = learned.LearnedProposal(G, Wt, M40, eps=0.01, seed=11, normalize=True)
        losses = lp.fit(n_labels=10**6, epochs=8, batch=8192, lr=3e-3, label_cap=64.0)
        margin = 1.2
    losses = losses.cpu().numpy()
    assert np.all(np.isfinite(losses))
    lp.build_proposal()
    assert lp.proposal.status() == 0
    mp, mi = lp.pilot(10**7, 0x5EED)
    ratio = mp.var / mi.var
    print(f"{variant}: variance ratio (method / learned) = {ratio:.3f}")
    z = (mp.estimate - mi.estimate) / math.sqrt(mp.stderr ** 2 + mi.stderr ** 2)
    assert abs(z) < 5.0
    assert ratio > margin
