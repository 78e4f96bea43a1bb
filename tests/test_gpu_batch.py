"""GPU tests of the batched sampler: several deltas and the six spine-sharing
motifs in one launch sequence.  Each delta's result must equal, bit for bit,
a single-delta call with the same (seed, stream, i0) and the oracle; results
must not depend on the tuning; the sequence must replay correctly from a
captured HIP graph; and the autotuner must return a usable tuning."""
import numpy as np
import pytest

import synthgraph as sg
from test_gpu_parity import _u64, build_both, check_sample

pytestmark = pytest.mark.gpu

SIX = [sg.MOTIFS[n] for n in sg.SIX_MOTIFS]
DELTAS = [600, 3600, 20000, 86400]


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
    Ws = [tcb.tc_path_weights(G, d) for d in DELTAS]
    return g, G, og, Ws


def same_result(a, b, per_sample=True):
    assert a.counts() == b.counts()
    assert np.array_equal(_u64(a.hits), _u64(b.hits))
    assert np.array_equal(a.estimate.cpu().numpy().view(np.uint64),
                          b.estimate.cpu().numpy().view(np.uint64))
    assert int(a.status.item()) == int(b.status.item())
    if per_sample:
        for f in ("e1", "e2", "e3"):
            assert np.array_equal(getattr(a, f).cpu().numpy(), getattr(b, f).cpu().numpy()), f
        assert np.array_equal(_u64(a.X), _u64(b.X))


def test_batch_equals_single_delta_calls_and_oracle(tcb, tiny):
    g, G, og, Ws = tiny
    k, seed, stream, i0 = 60000, 5, 3, 1000
    outs = tcb.tc_batch_estimate(G, Ws, SIX, k, seed, stream, i0, per_sample=True)
    mb = [sg.motif_bytes(M) for M in SIX]
    for d, delta in enumerate(DELTAS):
        single = tcb.tc_sample_estimate(G, Ws[d], SIX, k, seed, stream, i0, per_sample=True)
        same_result(outs[d], single)
        E = og.sample(og.weights(delta), mb, k, seed, stream, i0, per_sample=True)
        assert outs[d].counts() == E.cnt
        assert np.array_equal(_u64(outs[d].X), E.X)
        assert np.array_equal(outs[d].estimate.cpu().numpy().view(np.uint64),
                              E.est.view(np.uint64))


TUNINGS = [
    dict(chunk_log2=12, path_blocks=0, reg_waves=5120, fast_waves=5120, wide_blocks=1024),
    dict(chunk_log2=16, path_blocks=7, reg_waves=64, fast_waves=64, wide_blocks=64,
         reg_list_cap=128, lds_list_cap=256),
    dict(chunk_log2=25, path_blocks=1, reg_waves=100, fast_waves=16384, wide_blocks=2048,
         reg_list_cap=256, lds_list_cap=512),
    dict(chunk_log2=10, path_blocks=3000, reg_waves=1, fast_waves=1, wide_blocks=1,
         reg_list_cap=1, lds_list_cap=1),
]


@pytest.mark.parametrize("tuning", TUNINGS)
def test_batch_results_independent_of_tuning(tcb, tiny, tuning):
    g, G, og, Ws = tiny
    k = 40000
    ref = tcb.tc_batch_estimate(G, Ws, SIX, k, 9, per_sample=True)
    got = tcb.tc_batch_estimate(G, Ws, SIX, k, 9, per_sample=True,
                                tuning=tcb.make_tuning(**tuning))
    for a, b in zip(ref, got):
        same_result(a, b)


def test_chunk_beyond_2e22_samples(tcb, tiny):
    """One chunk holding all 5*10^6 samples of each delta (item codes with
    sample indices past 2^22) gives the counts, hits and estimates of
    2^15-sample chunks."""
    g, G, og, _ = tiny
    Ws = tcb.tc_path_weights_batch(G, [3600, 40000])
    k = 5_000_000
    big = tcb.tc_batch_estimate(G, Ws, SIX, k, 21, tuning=tcb.make_tuning(chunk_log2=25))
    small = tcb.tc_batch_estimate(G, Ws, SIX, k, 21, tuning=tcb.make_tuning(chunk_log2=16))
    for a, b in zip(big, small):
        assert int(a.status.item()) == int(b.status.item()) == 0
        assert a.counts() == b.counts()
        assert np.array_equal(_u64(a.hits), _u64(b.hits))
        assert np.array_equal(a.estimate.cpu().numpy().view(np.uint64),
                              b.estimate.cpu().numpy().view(np.uint64))
    assert sum(sum(r.counts()) for r in big) > 0


@pytest.fixture(scope="module")
def mid_lists(tcb, torch_mod):
    """The spine A->B->C->D (30 x 1 x 30 copies) and list pairs A->D, B->D
    whose windows hold about 60..800 entries: with the list caps of the
    tunings above, items move between the register tier (up to 128 or 256
    entries), the one-wavefront LDS tier (up to 256..1024) and the merged
    block-per-item tier."""
    rng = np.random.default_rng(77)
    A_, B_, C_, D_ = 0, 1, 2, 3
    src = [A_] * 30 + [B_] + [C_] * 30
    dst = [B_] * 30 + [C_] + [D_] * 30
    t = list(range(1, 31)) + [40] + list(range(41, 71))
    n_ad, n_bd, span = 1200, 500, 3000
    src += [A_] * n_ad + [B_] * n_bd
    dst += [D_] * (n_ad + n_bd)
    t += (100 + rng.integers(0, span, size=n_ad + n_bd)).tolist()
    g = sg.TemporalGraph(4, np.array(src, np.int32), np.array(dst, np.int32),
                         np.array(t, np.int64))
    G, og = build_both(tcb, torch_mod, g)
    motif = [(A_, B_), (B_, C_), (C_, D_), (A_, D_), (B_, D_), (A_, D_)]
    Ws = [tcb.tc_path_weights(G, d) for d in (400, 1000, 2500)]
    return G, og, [motif, motif[:5], motif[:4]], Ws


@pytest.mark.parametrize("tuning", TUNINGS)
def test_list_caps_route_items_without_changing_results(tcb, mid_lists, tuning):
    G, og, motifs, Ws = mid_lists
    k = 6000
    got = tcb.tc_batch_estimate(G, Ws, motifs, k, 13, per_sample=True,
                                tuning=tcb.make_tuning(**tuning))
    for d, W in enumerate(Ws):
        ref = tcb.tc_sample_estimate(G, W, motifs, k, 13, per_sample=True)
        same_result(got[d], ref)
    # and the default launch shape against the oracle, at the widest delta
    mb = [sg.motif_bytes(M) for M in motifs]
    E = og.sample(og.weights(2500), mb, k, 13, per_sample=True)
    assert got[2].counts() == E.cnt
    assert np.array_equal(_u64(got[2].X), E.X)


def test_batch_max_deltas_and_subsets(tcb, tiny):
    g, G, og, Ws = tiny
    extra = [tcb.tc_path_weights(G, d) for d in (0, 1, 7200, 10**6)]
    W8 = Ws + extra
    k = 20000
    outs = tcb.tc_batch_estimate(G, W8, SIX, k, 2, per_sample=True)
    for d in (0, 3, 4, 7):
        same_result(outs[d], tcb.tc_sample_estimate(G, W8[d], SIX, k, 2, per_sample=True))
    # one motif, two deltas (the single-motif launch shape)
    two = tcb.tc_batch_estimate(G, Ws[1:3], SIX[:1], k, 2, per_sample=True)
    for d in range(2):
        same_result(two[d], tcb.tc_sample_estimate(G, Ws[1 + d], SIX[:1], k, 2, per_sample=True))


def test_batch_planted_micro(tcb, torch_mod):
    import oracle  # noqa: F401
    g = sg.gen_micro_planted(3, SIX[3], copies=3, n=7, noise=12)
    G, og = build_both(tcb, torch_mod, g)
    Ws = [tcb.tc_path_weights(G, d) for d in (3, 9, 40)]
    outs = tcb.tc_batch_estimate(G, Ws, SIX, 20000, 4, per_sample=True)
    for d, delta in enumerate((3, 9, 40)):
        same_result(outs[d], check_sample(tcb, G, Ws[d], og, og.weights(delta), SIX, 20000,
                                          seed=4)[0])


def test_batch_argument_errors(tcb, tiny, torch_mod):
    g, G, og, Ws = tiny
    with pytest.raises(tcb.TCError):
        tcb.tc_batch_estimate(G, [], SIX, 100, 1)
    with pytest.raises(tcb.TCError):
        tcb.tc_batch_estimate(G, Ws + Ws + Ws[:1], SIX, 100, 1)  # 9 deltas
    small = torch_mod.empty(16, dtype=torch_mod.uint8, device="cuda")
    with pytest.raises(tcb.TCError) as e:
        tcb.tc_batch_estimate(G, Ws, SIX, 100, 1, workspace=small)
    assert e.value.code == tcb.TC_E_WORKSPACE


def test_batch_graph_capture_replays(tcb, tiny, torch_mod):
    """The whole batched sequence captured once, replayed three times with
    eager work in between (outputs poisoned before each replay); every replay
    must reproduce the eager result bit for bit."""
    torch = torch_mod
    g, G, og, Ws = tiny
    k, seed = 50000, 13
    eager = tcb.tc_batch_estimate(G, Ws, SIX, k, seed, per_sample=True)
    torch.cuda.synchronize()
    dev = G.ws.device
    outs = [tcb.new_result(len(SIX), k, dev, per_sample=True) for _ in Ws]
    ws = torch.empty(tcb.batch_workspace_bytes(k, len(Ws), len(SIX)), dtype=torch.uint8,
                     device=dev)
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph, stream=side):
        tcb.tc_batch_estimate(G, Ws, SIX, k, seed, outs=outs, workspace=ws)
    torch.cuda.synchronize()
    for rep in range(3):
        for o in outs:
            o.cnt.fill_(-1)
            o.hits.fill_(-1)
            o.estimate.fill_(float("nan"))
            o.status.fill_(-1)
            o.X.fill_(-7)
            o.e1.fill_(-3)
        ws.fill_(0xA5)
        torch.cuda.synchronize()
        graph.replay()
        torch.cuda.synchronize()
        for a, b in zip(outs, eager):
            same_result(a, b)


@pytest.mark.parametrize("wide", [False, True])
def test_whole_path_graph_capture_replays(tcb, torch_mod, wide):
    """Build, weights and sampling captured together in one HIP graph (the
    build enqueues a fixed launch sequence and waits for nothing), replayed
    three times with every workspace and output poisoned in between; each
    replay must give the graph arrays, S and the sampled results of the
    eager calls bit for bit.  `wide` takes a time range over 2^32, whose
    high-word sort passes are switched on by the device."""
    torch = torch_mod
    g = sg.gen_tiny()
    if wide:
        g.t = g.t * (2**20) - 2**40
    delta = 20000 * (2**20 if wide else 1)
    k, seed = 30000, 21
    s, d, t = (torch.from_numpy(g.src).cuda(), torch.from_numpy(g.dst).cuda(),
               torch.from_numpy(g.t).cuda())
    G = tcb.tc_build_graph(g.n, s, d, t, check=True)
    W = tcb.tc_path_weights(G, delta)
    R = tcb.tc_sample_estimate(G, W, SIX, k, seed, per_sample=True)
    torch.cuda.synchronize()
    R.check()
    dev = s.device
    ws_g = torch.empty(tcb.graph_workspace_bytes(g.n, g.m), dtype=torch.uint8, device=dev)
    ws_w = torch.empty(tcb.weights_workspace_bytes(g.m), dtype=torch.uint8, device=dev)
    ws_s = torch.empty(tcb.sample_workspace_bytes(k, len(SIX)), dtype=torch.uint8, device=dev)
    out = tcb.new_result(len(SIX), k, dev, per_sample=True)
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph, stream=side):
        G2 = tcb.tc_build_graph(g.n, s, d, t, workspace=ws_g)
        W2 = tcb.tc_path_weights(G2, delta, workspace=ws_w)
        tcb.tc_sample_estimate(G2, W2, SIX, k, seed, out=out, workspace=ws_s)
    torch.cuda.synchronize()
    ref_g = {kk: v.cpu() for kk, v in G.arrays().items()}
    ref_S = _u64(W.arrays()["S"])
    for rep in range(3):
        for buf in (ws_g, ws_w, ws_s):
            buf.fill_(0xA5)
        out.cnt.fill_(-1)
        out.estimate.fill_(float("nan"))
        out.status.fill_(-1)
        out.X.fill_(-7)
        out.e1.fill_(-3)
        # unrelated eager work between replays
        tcb.tc_path_weights(G, delta + 1)
        torch.cuda.synchronize()
        graph.replay()
        torch.cuda.synchronize()
        assert G2.status() == 0
        for kk, v in G2.arrays().items():
            assert torch.equal(v.cpu(), ref_g[kk]), kk
        assert G2.time_range() == G.time_range()
        assert np.array_equal(_u64(W2.arrays()["S"]), ref_S)
        same_result(out, R)


def test_autotune_returns_usable_tuning(tcb, tiny):
    g, G, og, Ws = tiny
    best, ms = tcb.tc_autotune(G, Ws, SIX, 100000, seed=1)
    t = best.as_dict()
    assert 10 <= t["chunk_log2"] <= 25 and ms > 0
    assert t["reg_waves"] >= 1 and t["fast_waves"] >= 1 and t["path_blocks"] >= 0
    ref = tcb.tc_batch_estimate(G, Ws, SIX, 30000, 3, per_sample=True)
    got = tcb.tc_batch_estimate(G, Ws, SIX, 30000, 3, per_sample=True, tuning=best)
    for a, b in zip(ref, got):
        same_result(a, b)
