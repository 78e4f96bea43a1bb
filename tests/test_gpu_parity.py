"""GPU parity: the HIP path through the C ABI against the CPU oracle on the
same seeded inputs.  Integer work (orders, offsets, window metadata, S, the
sampled paths, X, cnt, hits) must match bit for bit; the FP64 estimate is
checked to 1e-9 relative and is expected to be bit-identical (both sides
round each integer to nearest binary64 and then divide and multiply)."""
import math

import numpy as np
import pytest

import synthgraph as sg

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


def _u64(t):
    return t.cpu().numpy().view(np.uint64)


def _u32(t):
    return t.cpu().numpy().view(np.uint32)


def _dev(torch, g):
    return (torch.from_numpy(g.src).cuda(), torch.from_numpy(g.dst).cuda(),
            torch.from_numpy(g.t).cuda())


def build_both(tcb, torch, g):
    import oracle
    s, d, t = _dev(torch, g)
    G = tcb.tc_build_graph(g.n, s, d, t)
    og = oracle.OracleGraph.from_graph(g)
    return G, og


def check_graph(G, og, g):
    assert G.status() == 0
    A = G.arrays()
    o = og.orders()
    assert np.array_equal(A["out_eid"].cpu().numpy(), o["out_eid"])
    assert np.array_equal(A["in_eid"].cpu().numpy(), o["in_eid"])
    assert np.array_equal(A["pair_eid"].cpu().numpy(), o["pair_eid"])
    assert np.array_equal(_u32(A["out_off"]), o["out_off"])
    assert np.array_equal(_u32(A["in_off"]), o["in_off"])
    oe, ie, pe = o["out_eid"], o["in_eid"], o["pair_eid"]
    assert np.array_equal(A["out_src"].cpu().numpy(), g.src[oe])
    assert np.array_equal(A["out_dst"].cpu().numpy(), g.dst[oe])
    assert np.array_equal(A["out_t"].cpu().numpy(), g.t[oe])
    assert np.array_equal(A["in_src"].cpu().numpy(), g.src[ie])
    assert np.array_equal(A["in_t"].cpu().numpy(), g.t[ie])
    assert np.array_equal(A["pair_dst"].cpu().numpy(), g.dst[pe])
    assert np.array_equal(A["pair_t"].cpu().numpy(), g.t[pe])
    # 16-byte records {other end, eid, t} of the two CSRs
    m = g.m
    if m:
        orec = G.view("out_rec", torch_i32(), 4 * m).cpu().numpy().reshape(m, 4)
        irec = G.view("in_rec", torch_i32(), 4 * m).cpu().numpy().reshape(m, 4)
        assert np.array_equal(orec[:, 0], g.dst[oe]) and np.array_equal(orec[:, 1], oe)
        assert np.array_equal(orec[:, 2:].copy().view(np.int64).ravel(), g.t[oe])
        assert np.array_equal(irec[:, 0], g.src[ie]) and np.array_equal(irec[:, 1], ie)
        assert np.array_equal(irec[:, 2:].copy().view(np.int64).ravel(), g.t[ie])


def torch_i32():
    import torch
    return torch.int32


def check_weights(Wt, ow, g=None, og=None):
    A = Wt.arrays()
    assert np.array_equal(_u32(A["lo_in"]), ow.lo_in)
    assert np.array_equal(_u32(A["a"]), ow.a)
    assert np.array_equal(_u32(A["lo_out"]), ow.lo_out)
    assert np.array_equal(_u32(A["b"]), ow.b)
    assert np.array_equal(_u64(A["S"]), ow.S)
    assert Wt.status() == ow.status
    m = ow.a.shape[0]
    if m:
        # 32-byte path records {lo_in, a, lo_out, b, u, v, t}
        pr = Wt.view("prec", torch_i32(), 8 * m).cpu().numpy().reshape(m, 8)
        assert np.array_equal(pr[:, 0].view(np.uint32), ow.lo_in)
        assert np.array_equal(pr[:, 1].view(np.uint32), ow.a)
        assert np.array_equal(pr[:, 2].view(np.uint32), ow.lo_out)
        assert np.array_equal(pr[:, 3].view(np.uint32), ow.b)
        if g is not None:
            oe = og.orders()["out_eid"]
            assert np.array_equal(pr[:, 4], g.src[oe]) and np.array_equal(pr[:, 5], g.dst[oe])
            assert np.array_equal(pr[:, 6:].copy().view(np.int64).ravel(), g.t[oe])


def check_sample(tcb, G, Wt, og, ow, motifs, k, seed, stream=0, i0=0, per_sample=True):
    mb = [sg.motif_bytes(M) for M in motifs]
    R = tcb.tc_sample_estimate(G, Wt, motifs, k, seed, stream, i0, per_sample=per_sample)
    E = og.sample(ow, mb, k, seed, stream, i0, per_sample=per_sample)
    st = int(R.status.item()) & 0xFFFFFFFF
    assert st == E.status, (st, E.status)
    if per_sample:
        assert np.array_equal(R.e1.cpu().numpy(), E.e1)
        assert np.array_equal(R.e2.cpu().numpy(), E.e2)
        assert np.array_equal(R.e3.cpu().numpy(), E.e3)
        assert np.array_equal(_u64(R.X), E.X)
    if st == 0:
        assert R.counts() == E.cnt
        assert np.array_equal(_u64(R.hits), E.hits)
        est = R.estimate.cpu().numpy()
        for j in range(len(motifs)):
            assert est[j] == E.est[j] or abs(est[j] - E.est[j]) <= 1e-9 * abs(E.est[j])
        assert np.array_equal(est.view(np.uint64), E.est.view(np.uint64))
    return R, E


# ----------------------------------------------------------------- tiny ----
@pytest.fixture(scope="module")
def tiny(tcb, torch_mod):
    g = sg.gen_tiny()
    G, og = build_both(tcb, torch_mod, g)
    return g, G, og


def test_tiny_graph_orders(tiny):
    g, G, og = tiny
    check_graph(G, og, g)


def test_pair_skip_levels(tcb, tiny, torch_mod):
    """The sampled levels of the pair times used by the searches inside a
    run are pair_t[16^k i] for k = 1, 2, 3."""
    g, G, og = tiny
    # sampled levels of the pair times used by the searches inside a run
    pt = G.arrays()["pair_t"].cpu().numpy()
    n = [-(-g.m // 16 ** k) for k in (1, 2, 3)]
    skip = G.view("pair_skip", torch_mod.int64, sum(n)).cpu().numpy()
    assert np.array_equal(skip[:n[0]], pt[::16])
    assert np.array_equal(skip[n[0]:n[0] + n[1]], pt[::256])
    assert np.array_equal(skip[n[0] + n[1]:], pt[::4096])


@pytest.mark.parametrize("delta", [0, 3600, 20000, 10**6])
def test_tiny_weights(tcb, tiny, delta):
    g, G, og = tiny
    Wt = tcb.tc_path_weights(G, delta)
    check_weights(Wt, og.weights(delta), g, og)


def test_tiny_m40_k1e5_seed1(tcb, tiny):
    """The tiny workload as specified: delta 3,600, M4-0, k = 10^5, seed 1."""
    g, G, og = tiny
    Wt = tcb.tc_path_weights(G, 3600)
    ow = og.weights(3600)
    R, E = check_sample(tcb, G, Wt, og, ow, [M40], 10**5, seed=1)
    C = og.brute_count(sg.motif_bytes(M40), 3600)
    assert C > 0 and R.counts()[0] > 0


@pytest.mark.parametrize("delta,seed,stream", [(20000, 3, 0), (86400, 7, 5), (3600, 2**40 + 9, 2**31)])
def test_tiny_six_motifs(tcb, tiny, delta, seed, stream):
    g, G, og = tiny
    Wt = tcb.tc_path_weights(G, delta)
    ow = og.weights(delta)
    check_sample(tcb, G, Wt, og, ow, SIX, 50000, seed=seed, stream=stream)


def test_tiny_chunked_equals_one_shot(tcb, tiny):
    g, G, og = tiny
    Wt = tcb.tc_path_weights(G, 20000)
    full = tcb.tc_sample_estimate(G, Wt, SIX, 30000, 4, 1, 0, per_sample=True)
    parts = [tcb.tc_sample_estimate(G, Wt, SIX, 10000, 4, 1, i0, per_sample=True)
             for i0 in (0, 10000, 20000)]
    for j in range(len(SIX)):
        assert full.counts()[j] == sum(p.counts()[j] for p in parts)
    assert np.array_equal(_u64(full.X), np.concatenate([_u64(p.X) for p in parts], axis=1))


def test_determinism_repeat_runs(tcb, tiny):
    g, G, og = tiny
    Wt = tcb.tc_path_weights(G, 20000)
    a = tcb.tc_sample_estimate(G, Wt, SIX, 100000, 11)
    b = tcb.tc_sample_estimate(G, Wt, SIX, 100000, 11)
    assert a.counts() == b.counts()
    assert np.array_equal(a.estimate.cpu().numpy(), b.estimate.cpu().numpy())


def test_counter_high_word_crossed(tcb, tiny):
    """Samples i0 .. i0 + k - 1 straddle i = 2^32: the Philox counter's
    second word changes inside the call."""
    g, G, og = tiny
    Wt = tcb.tc_path_weights(G, 20000)
    ow = og.weights(20000)
    i0 = (1 << 32) - 1000
    check_sample(tcb, G, Wt, og, ow, SIX, 2000, seed=5, stream=3, i0=i0)
    # and far above: the high word well past zero
    check_sample(tcb, G, Wt, og, ow, SIX, 1500, seed=6, stream=0, i0=(1 << 40) + 77)


def test_wide_vertex_ids_26_bits(tcb, torch_mod):
    """Vertex ids spread over [0, 2^26): 26-bit keys take three radix passes
    of 8, 9 and 9 bits per vertex sort and the offset arrays have 2^26 + 1
    entries."""
    g = sg.relabel_spread(sg.gen_tiny(), 1 << 26, seed=41)
    G, og = build_both(tcb, torch_mod, g)
    check_graph(G, og, g)
    Wt = tcb.tc_path_weights(G, 20000)
    ow = og.weights(20000)
    check_weights(Wt, ow, g, og)
    check_sample(tcb, G, Wt, og, ow, SIX, 40000, seed=2)


@pytest.mark.parametrize("n_new", [512, 1 << 17, 1 << 25])
def test_nine_bit_digit_sorts(tcb, torch_mod, n_new):
    """Vertex-id widths at which 9-bit digits save a radix pass (9, 17 and 25
    bits: one, two and three passes over 512-entry digit histograms), on an
    edge list of nine tiles with a ragged tail."""
    g = sg.gen_micro(12289, n=512, m=12289, t_span=6000)
    if n_new > g.n:
        g = sg.relabel_spread(g, n_new, seed=n_new % 97)
    G, og = build_both(tcb, torch_mod, g)
    check_graph(G, og, g)
    Wt = tcb.tc_path_weights(G, 600)
    ow = og.weights(600)
    check_weights(Wt, ow, g, og)
    check_sample(tcb, G, Wt, og, ow, SIX, 3000, seed=n_new % 89)


@pytest.mark.parametrize("tbits", [9, 10, 13, 18, 20, 28, 30, 33, 41, 50])
def test_time_sort_digit_widths(tcb, torch_mod, tbits):
    """Time ranges of exactly tbits bits (from negative times up): two to
    four passes over the low word, with high-word passes past 32 bits, digit
    widths from 1 to 8 bits; nine tiles with a ragged tail and many ties."""
    base = sg.gen_micro(12289 + tbits, n=300, m=12289, t_span=4000)
    t = base.t.astype(np.int64)
    span = max(1, int(t.max() - t.min()))
    t = (t - t.min()) * ((1 << tbits) - 1) // span - (1 << (tbits - 1))
    g = sg.TemporalGraph(base.n, base.src, base.dst, t, name="tbits%d" % tbits)
    assert int(t.max() - t.min()).bit_length() == tbits
    G, og = build_both(tcb, torch_mod, g)
    check_graph(G, og, g)
    delta = 1 << (tbits - 5)
    Wt = tcb.tc_path_weights(G, delta)
    ow = og.weights(delta)
    check_weights(Wt, ow, g, og)
    check_sample(tcb, G, Wt, og, ow, SIX, 2000, seed=tbits)


# --------------------------------------------------- micro / edge cases ----
@pytest.mark.parametrize("seed", range(6))
def test_planted_micro(tcb, torch_mod, seed):
    M = SIX[seed % len(SIX)]
    g = sg.gen_micro_planted(seed, M, copies=3, n=7, noise=12)
    G, og = build_both(tcb, torch_mod, g)
    check_graph(G, og, g)
    for delta in (3, 9, 40):
        Wt = tcb.tc_path_weights(G, delta)
        ow = og.weights(delta)
        check_weights(Wt, ow, g, og)
        check_sample(tcb, G, Wt, og, ow, SIX, 20000, seed=seed + 1)


@pytest.mark.parametrize("m", [1, 2, 63, 2047, 2049, 4095, 4096, 4097, 12289])
def test_ragged_sizes(tcb, torch_mod, m):
    g = sg.gen_micro(m, n=max(3, m // 8), m=m, t_span=max(4, m // 2))
    G, og = build_both(tcb, torch_mod, g)
    check_graph(G, og, g)
    delta = max(2, m // 10)
    Wt = tcb.tc_path_weights(G, delta)
    ow = og.weights(delta)
    check_weights(Wt, ow, g, og)
    check_sample(tcb, G, Wt, og, ow, SIX, 3000, seed=m)


def test_empty_graph(tcb, torch_mod):
    e32 = torch_mod.zeros(0, dtype=torch_mod.int32, device="cuda")
    e64 = torch_mod.zeros(0, dtype=torch_mod.int64, device="cuda")
    G = tcb.tc_build_graph(5, e32, e32, e64)
    assert G.m == 0
    assert (G.arrays()["out_off"].cpu() == 0).all()
    Wt = tcb.tc_path_weights(G, 10)
    assert Wt.total() == 0 and Wt.status() == 0
    R = tcb.tc_sample_estimate(G, Wt, SIX, 100, 1, per_sample=True)
    R.check()
    assert R.counts() == [0] * 6 and (R.estimate.cpu() == 0).all()
    assert (R.e1.cpu() == -1).all() and (R.X.cpu() == 0).all()


def test_zero_weight_graph(tcb, torch_mod):
    src = np.array([0, 2], np.int32)
    dst = np.array([1, 3], np.int32)
    t = np.array([5, 6], np.int64)
    g = sg.TemporalGraph(4, src, dst, t)
    G, og = build_both(tcb, torch_mod, g)
    Wt = tcb.tc_path_weights(G, 100)
    ow = og.weights(100)
    check_weights(Wt, ow, g, og)
    check_sample(tcb, G, Wt, og, ow, [M40], 257, seed=1)


def test_single_vertex_and_wide_time_range(tcb, torch_mod):
    # n = 1: every edge is a self-loop (in the CSR and W, never a match)
    g = sg.TemporalGraph(1, np.zeros(50, np.int32), np.zeros(50, np.int32),
                         np.arange(50, dtype=np.int64) % 7)
    G, og = build_both(tcb, torch_mod, g)
    check_graph(G, og, g)
    Wt = tcb.tc_path_weights(G, 3)
    ow = og.weights(3)
    check_weights(Wt, ow, g, og)
    check_sample(tcb, G, Wt, og, ow, [M40], 1000, seed=2)
    # timestamps spanning more than 32 bits (64-bit radix keys), negatives
    rng = np.random.default_rng(5)
    g = sg.gen_micro(9, n=6, m=3000, t_span=10)
    g.t = (g.t - 5) * (2**58) + rng.integers(-3, 4, size=g.m)
    G, og = build_both(tcb, torch_mod, g)
    check_graph(G, og, g)
    for delta in (0, 2**58, 2**62):
        Wt = tcb.tc_path_weights(G, delta)
        ow = og.weights(delta)
        check_weights(Wt, ow, g, og)
        check_sample(tcb, G, Wt, og, ow, SIX, 5000, seed=3)


def test_equal_timestamps(tcb, torch_mod):
    # one timestamp for every edge: the time sort has no pass, so its re-keying
    # of the records for the next two sorts runs on its own
    g = sg.gen_micro(21, n=40, m=5000, t_span=10)
    g.t = np.full(g.m, 123456789, np.int64)
    G, og = build_both(tcb, torch_mod, g)
    check_graph(G, og, g)
    for delta in (0, 5):
        Wt = tcb.tc_path_weights(G, delta)
        ow = og.weights(delta)
        check_weights(Wt, ow, g, og)
        check_sample(tcb, G, Wt, og, ow, SIX, 3000, seed=4)


def test_range_errors(tcb, torch_mod):
    """A bad vertex id or time is reported in the build's device status word;
    the weights of such a graph carry TC_F_RANGE with W = 0 and the sampler
    draws nothing (no kernel reads through the unsorted arrays)."""
    cases = [([0, 1], [1, 3], [0, 1]),            # dst == n
             ([0, -1], [1, 2], [0, 1]),           # negative id
             ([0, 1], [1, 2], [0, 2**62]),        # |t| = 2^62
             ([0, 1], [1, 2], [-(2**62), 5])]
    for s_, d_, t_ in cases:
        s = torch_mod.tensor(s_, dtype=torch_mod.int32, device="cuda")
        d = torch_mod.tensor(d_, dtype=torch_mod.int32, device="cuda")
        t = torch_mod.tensor(t_, dtype=torch_mod.int64, device="cuda")
        G = tcb.tc_build_graph(3, s, d, t)
        assert G.status() == tcb.TC_F_RANGE
        with pytest.raises(tcb.TCDeviceError):
            G.check()
        with pytest.raises(tcb.TCDeviceError):
            tcb.tc_build_graph(3, s, d, t, check=True)
        Wt = tcb.tc_path_weights(G, 10)
        assert Wt.status() == tcb.TC_F_RANGE and Wt.total() == 0
        R = tcb.tc_sample_estimate(G, Wt, SIX, 1000, 1, per_sample=True)
        assert (int(R.status.item()) & tcb.TC_F_RANGE) != 0
        assert R.counts() == [0] * 6
    s = torch_mod.tensor([0, 1], dtype=torch_mod.int32, device="cuda")
    d = torch_mod.tensor([1, 2], dtype=torch_mod.int32, device="cuda")
    t = torch_mod.tensor([-(2**62) + 1, 2**62 - 1], dtype=torch_mod.int64, device="cuda")
    G = tcb.tc_build_graph(3, s, d, t, check=True)
    assert G.time_range() == (-(2**62) + 1, 2**62 - 1)


def test_weight_overflow(tcb, torch_mod):
    g = sg.gen_overflow_layers(2**21, 2**22, 2**21)
    G, og = build_both(tcb, torch_mod, g)
    Wt = tcb.tc_path_weights(G, 0)
    assert Wt.status() == tcb.TC_F_OVERFLOW
    R = tcb.tc_sample_estimate(G, Wt, [M40], 1000, 1)
    with pytest.raises(tcb.TCDeviceError):
        R.check()
    del G, og
    g = sg.gen_overflow_layers(2**21, 2**22 - 1, 2**21)
    G, og = build_both(tcb, torch_mod, g)
    Wt = tcb.tc_path_weights(G, 0)
    ow = og.weights(0)
    assert Wt.status() == 0 and Wt.total() == 2**64 - 2**42
    check_weights(Wt, ow, g, og)
    check_sample(tcb, G, Wt, og, ow, [M40], 20000, seed=1)


def test_listcount_counts_beyond_2e64(tcb, torch_mod):
    """A 16-edge motif (13 lists, the most the descriptor allows) with 32
    edges per list in disjoint increasing time blocks: every draw of one of
    the 64*64 planted spines has 32^13 = 2^65 chains.  Such counts go to the
    128-bit ListCount pass: cnt is exact (its sum over samples, compared with
    the oracle's 128-bit arithmetic), the per-sample X saturates at 2^64 - 1,
    and nothing is flagged."""
    A_, B_, C_, D_ = 0, 1, 2, 3
    ranks = [(D_, A_), (A_, C_), (B_, D_), (D_, C_), (C_, B_), (B_, A_), (A_, D_), (C_, A_),
             (D_, B_), (A_, B_), (B_, C_), (C_, D_), (D_, A_)]
    motif = [(A_, B_), (B_, C_), (C_, D_)] + ranks
    p = q = 64
    src = [A_] * p + [B_] + [C_] * q
    dst = [B_] * p + [C_] + [D_] * q
    t = list(range(1, p + 1)) + [p + 1] + list(range(p + 2, p + q + 2))
    base = 1000
    for (a, b) in ranks:
        src += [a] * 32
        dst += [b] * 32
        t += list(range(base, base + 32))
        base += 64
    g = sg.TemporalGraph(4, np.array(src, np.int32), np.array(dst, np.int32),
                         np.array(t, np.int64))
    G, og = build_both(tcb, torch_mod, g)
    delta = base + 10
    Wt = tcb.tc_path_weights(G, delta)
    ow = og.weights(delta)
    check_weights(Wt, ow, g, og)
    R, E = check_sample(tcb, G, Wt, og, ow, [motif], 20000, seed=1, per_sample=True)
    assert E.status == 0
    hits = int(E.hits[0])
    assert hits > 0 and E.cnt[0] == hits * 32**13
    assert (E.X[0][E.X[0] != 0] == np.uint64(2**64 - 1)).all()
    # beside a motif with small counts: both exact
    R, E = check_sample(tcb, G, Wt, og, ow, [motif, M40], 20000, seed=1, per_sample=False)
    assert E.status == 0 and R.counts()[0] == E.cnt[0] > 2**64
    # the same graph with the 4-cycle only
    check_sample(tcb, G, Wt, og, ow, [M40, motif[:9]], 20000, seed=1, per_sample=True)
    # importance sampling cannot take a count of 2^64 or more: flagged
    h = torch_mod.full((g.m,), 2, dtype=torch_mod.int32, device="cuda")
    Wq = tcb.tc_proposal_weights(G, Wt, h)
    Rq = tcb.tc_sample_estimate(G, Wq, [motif, M40], 20000, 1)
    assert (int(Rq.status.item()) & 0xFFFFFFFF) == 2 | (1 << 8)


@pytest.mark.parametrize("per_block", [40, 200])
def test_long_lists_counts_beyond_2e64(tcb, torch_mod, per_block):
    """Counts beyond 2^64 from the LDS-key pass (lists of 280 entries) and
    from the merged pass (1,400): the planted spines A->B->C->D (64 x 1 x 64)
    and a motif with 13 lists alternating A->D and B->D, whose edges come in
    13 increasing time blocks of per_block edges (blocks alternate the two
    pairs).  D has no out-edges and A no in-edges, so W is the 4,096 spines
    and every draw is one of them; its chain count is above 2^64 (6.7e20 and
    8.2e29).  The 128-bit merged pass takes these items: cnt and the
    saturated X equal the oracle's, nothing is flagged."""
    A_, B_, C_, D_ = 0, 1, 2, 3
    n_lists = 13
    pairs = [(A_, D_) if r % 2 == 0 else (B_, D_) for r in range(n_lists)]
    motif = [(A_, B_), (B_, C_), (C_, D_)] + pairs
    p = q = 64
    src = [A_] * p + [B_] + [C_] * q
    dst = [B_] * p + [C_] + [D_] * q
    t = list(range(1, p + 1)) + [p + 1] + list(range(p + 2, p + q + 2))
    base = 1000
    for (a, b) in pairs:
        src += [a] * per_block
        dst += [b] * per_block
        t += list(range(base, base + per_block))
        base += per_block + 5
    g = sg.TemporalGraph(4, np.array(src, np.int32), np.array(dst, np.int32),
                         np.array(t, np.int64))
    G, og = build_both(tcb, torch_mod, g)
    delta = base + 10
    Wt = tcb.tc_path_weights(G, delta)
    ow = og.weights(delta)
    assert Wt.total() == p * q
    k = 6000
    R, E = check_sample(tcb, G, Wt, og, ow, [motif], k, seed=3, per_sample=True)
    assert E.status == 0 and int(E.hits[0]) == k
    assert E.cnt[0] > k * 2**64
    assert (E.X[0] == np.uint64(2**64 - 1)).all()
    R, E = check_sample(tcb, G, Wt, og, ow, [M40, motif], k, seed=4, per_sample=False)
    assert E.status == 0 and R.counts()[1] == E.cnt[1] > 2**64


LONG_CASES = {
    # name: (A->D edges, B->D edges, time span of the lists, delta offset)
    "wide_balanced": (3000, 2000, 4000, 0),
    "wide_imbalanced": (60, 90000, 30000, 0),
    "wide_ragged": (2100, 2000, 1500, 0),
    "wide_delta_2e32": (900, 700, 1200, 2**33),
    "big": (150000, 400, 20000, 0),
}


@pytest.mark.parametrize("case", list(LONG_CASES))
def test_long_lists_tiers(tcb, torch_mod, case):
    """Items whose lists run past the register and LDS tiers: the spine
    A->B->C->D (30 x 1 x 30 copies, so every draw is this spine with its own
    t1 and t3) and a motif with three lists A->D, B->D, A->D after it.  D has
    no out-edges, so no list edge centres a path.  List times are drawn with
    many ties over `span` seconds and delta cuts through them, so the windows
    differ with t1; lengths reach the merged block-per-item tier (1,025 ..
    65,536 entries, with a strongly imbalanced pair and with delta >= 2^32)
    and the one-thread tier beyond."""
    n_ad, n_bd, span, dplus = LONG_CASES[case]
    A_, B_, C_, D_ = 0, 1, 2, 3
    rng = np.random.default_rng(len(case))
    src = [A_] * 30 + [B_] + [C_] * 30
    dst = [B_] * 30 + [C_] + [D_] * 30
    t = list(range(1, 31)) + [40] + list(range(41, 71))
    t0 = 100
    src += [A_] * n_ad + [B_] * n_bd
    dst += [D_] * (n_ad + n_bd)
    t += (t0 + rng.integers(0, span, size=n_ad)).tolist()
    t += (t0 + rng.integers(0, span, size=n_bd)).tolist()
    g = sg.TemporalGraph(4, np.array(src, np.int32), np.array(dst, np.int32),
                         np.array(t, np.int64))
    G, og = build_both(tcb, torch_mod, g)
    motif = [(A_, B_), (B_, C_), (C_, D_), (A_, D_), (B_, D_), (A_, D_)]
    delta = t0 + span // 2 + dplus
    Wt = tcb.tc_path_weights(G, delta)
    ow = og.weights(delta)
    check_weights(Wt, ow, g, og)
    assert ow.W == 900
    R, E = check_sample(tcb, G, Wt, og, ow, [motif, motif[:5]], 3000, seed=4, per_sample=True)
    assert E.status == 0 and int(E.hits[0]) > 0


# --------------------------------------------------------- medium scale ----
@pytest.fixture(scope="module")
def medium(tcb, torch_mod):
    g = sg.gen_medium()
    G, og = build_both(tcb, torch_mod, g)
    return g, G, og


def test_medium_full_size_parity(tcb, medium):
    """The medium workload at full size (10^6 vertices, 2*10^7 edges,
    delta 86,400, six motifs, k = 10^7) in the launch shape the benchmark
    times: orders, weights and all six counts compared in full, plus every
    per-sample output on a 2*10^5-sample window of the same stream."""
    g, G, og = medium
    check_graph(G, og, g)
    delta = sg.MEDIUM["delta"]
    Wt = tcb.tc_path_weights(G, delta)
    ow = og.weights(delta)
    check_weights(Wt, ow, g, og)
    check_sample(tcb, G, Wt, og, ow, SIX, sg.MEDIUM["k"], seed=1, per_sample=False)
    check_sample(tcb, G, Wt, og, ow, SIX, 200000, seed=1, i0=4_000_000, per_sample=True)
