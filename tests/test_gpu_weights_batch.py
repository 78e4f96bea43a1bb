"""GPU parity of the batched Preprocess (Algorithm Preprocess with Claim
"count", for several deltas of one anchor class at once): every weights set
of a tc_path_weights_batch call must equal, word for word, the oracle's
windows and S for its delta and what tc_path_weights_class gives for that
delta alone.  The cases reach every record width (one, two to three, four
to seven and eight deltas), every class, repeated deltas, delta = 0 and
2^62, ragged edge counts, a rejected graph and the 2^64 overflow."""
import numpy as np
import pytest

import synthgraph as sg
from test_gpu_parity import _u32, _u64, build_both, check_weights, M40

pytestmark = pytest.mark.gpu

PATH_CLASSES = [(m1, a1, m3, a3) for m1 in (1, 2) for a1 in (0, 1) for m3 in (1, 2)
                for a3 in (0, 1)]
WEDGE_CLASSES = [(m1, a1, 0, 0) for m1 in (1, 2) for a1 in (0, 1)] + \
                [(0, 0, m3, a3) for m3 in (1, 2) for a3 in (0, 1)]


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


def _words(W, m):
    """Every array a weights set owns, as bytes: windows, S, status and the
    path records."""
    A = W.arrays()
    out = {k: A[k].cpu().numpy().tobytes() for k in ("lo_in", "a", "lo_out", "b", "S")}
    out["status"] = W.status()
    if m:
        import torch
        out["prec"] = W.view("prec", torch.int32, 8 * m).cpu().numpy().tobytes()
    return out


def _same_as_single(tcb, G, Ws, deltas, cls, m):
    for W, d in zip(Ws, deltas):
        S1 = tcb.tc_path_weights(G, d, cls=cls)
        a, b = _words(W, m), _words(S1, m)
        assert a.keys() == b.keys()
        for k in a:
            assert a[k] == b[k], (d, cls, k)
        assert W.c.delta == d and W.c.cls.as_tuple() == tuple(cls)


@pytest.mark.parametrize("cls", PATH_CLASSES + WEDGE_CLASSES)
def test_batch_every_class_against_oracle(tcb, tiny, cls):
    g, G, og = tiny
    deltas = [0, 3600, 40000]
    Ws = tcb.tc_path_weights_batch(G, deltas, cls=cls)
    for W, d in zip(Ws, deltas):
        ow = og.weights(d, cls=bytes(cls))
        A = W.arrays()
        for name in ("lo_in", "a", "lo_out", "b"):
            assert np.array_equal(_u32(A[name]), getattr(ow, name)), (d, name)
        assert np.array_equal(_u64(A["S"]), ow.S)
        assert W.status() == ow.status
    _same_as_single(tcb, G, Ws, deltas, cls, g.src.size)


@pytest.mark.parametrize("deltas", [[3600], [0, 86400], [5, 5, 2**62],
                                    [1, 10, 100, 1000, 10**4, 10**5, 10**6],
                                    [2**62, 0, 7, 3600, 3600, 86400, 12345, 1]])
def test_batch_widths_spine(tcb, tiny, deltas):
    """One to eight deltas (records of 2, 4, 8 and 12 words), repeats, the
    extremes; the spine class's path records against the oracle too."""
    g, G, og = tiny
    Ws = tcb.tc_path_weights_batch(G, deltas)
    for W, d in zip(Ws, deltas):
        check_weights(W, og.weights(d), g, og)
    _same_as_single(tcb, G, Ws, deltas, (1, 0, 2, 1), g.src.size)


@pytest.mark.parametrize("m", [1, 2, 2047, 2048, 2049, 6145])
def test_batch_ragged_sizes(tcb, torch_mod, m):
    g = sg.gen_tiny(seed=77 + m, n=max(3, m // 3), m=m, t_max=5000)
    G, og = build_both(tcb, torch_mod, g)
    deltas = [0, 60, 600, 5000]
    for cls in [(1, 0, 2, 1), (2, 1, 1, 0), (0, 0, 2, 1), (1, 1, 0, 0)]:
        Ws = tcb.tc_path_weights_batch(G, deltas, cls=cls)
        for W, d in zip(Ws, deltas):
            ow = og.weights(d, cls=bytes(cls))
            A = W.arrays()
            for name in ("lo_in", "a", "lo_out", "b"):
                assert np.array_equal(_u32(A[name]), getattr(ow, name)), (m, cls, d, name)
            assert np.array_equal(_u64(A["S"]), ow.S)
        _same_as_single(tcb, G, Ws, deltas, cls, m)


def test_batch_feeds_the_sampler(tcb, tiny):
    """Batched weights drive the batched sampler to the oracle's results."""
    g, G, og = tiny
    deltas = [600, 3600, 86400]
    Ws = tcb.tc_path_weights_batch(G, deltas)
    outs = tcb.tc_batch_estimate(G, Ws, [M40], 20000, 9, per_sample=True)
    mb = [sg.motif_bytes(M40)]
    for R, d in zip(outs, deltas):
        E = og.sample(og.weights(d), mb, 20000, 9, 0, 0, per_sample=True)
        assert int(R.status.item()) & 0xFFFFFFFF == E.status
        assert np.array_equal(R.e2.cpu().numpy(), E.e2)
        assert np.array_equal(_u64(R.X), E.X)
        assert R.counts() == E.cnt


def test_batch_rejected_graph(tcb, torch_mod):
    s = torch_mod.tensor([0, 1, 2], dtype=torch_mod.int32, device="cuda")
    d = torch_mod.tensor([1, 3, 0], dtype=torch_mod.int32, device="cuda")
    t = torch_mod.tensor([0, 1, 2], dtype=torch_mod.int64, device="cuda")
    G = tcb.tc_build_graph(3, s, d, t)
    Ws = tcb.tc_path_weights_batch(G, [0, 10, 100])
    for W in Ws:
        assert W.status() == tcb.TC_F_RANGE and W.total() == 0


def test_batch_overflow(tcb, torch_mod):
    g = sg.gen_overflow_layers(2**21, 2**22, 2**21)
    G, og = build_both(tcb, torch_mod, g)
    Ws = tcb.tc_path_weights_batch(G, [0, 1, 2**40])
    for W in Ws:
        assert W.status() == tcb.TC_F_OVERFLOW
    del G, og, Ws
    g = sg.gen_overflow_layers(2**21, 2**22 - 1, 2**21)
    G, og = build_both(tcb, torch_mod, g)
    Ws = tcb.tc_path_weights_batch(G, [0, 3])
    for W, d in zip(Ws, [0, 3]):
        assert W.status() == 0 and W.total() == 2**64 - 2**42
        check_weights(W, og.weights(d), g, og)


def test_batch_host_errors(tcb, tiny):
    g, G, og = tiny
    for bad in ([], list(range(9)), [-1], [2**62 + 1]):
        with pytest.raises(tcb.TCError):
            tcb.tc_path_weights_batch(G, bad)
    with pytest.raises(tcb.TCError):
        tcb.tc_path_weights_batch(G, [1, 2], cls=(0, 0, 0, 0))


def _hub_graph(seed=5, per_side=12000, others=400, span=100000):
    """Two hubs with dense in- and out-lists (windows far wider than a rank
    tile and its staged neighbours at the larger deltas), edges between the
    hubs, and sparse noise."""
    rng = np.random.default_rng(seed)
    H, K = 0, 1
    x = rng.integers(2, 2 + others, size=per_side)
    y = rng.integers(2, 2 + others, size=per_side)
    ns = rng.integers(2, 2 + others, size=3000)
    nd = rng.integers(2, 2 + others, size=3000)
    src = np.concatenate([x, np.full(per_side, H), np.full(2000, H), np.full(2000, K), ns])
    dst = np.concatenate([np.full(per_side, H), y, np.full(2000, K), np.full(2000, H), nd])
    t = rng.integers(0, span, size=src.size)
    t[:50] = 777  # ties at one time
    keep = src != dst
    return sg.TemporalGraph(2 + others, src[keep].astype(np.int32), dst[keep].astype(np.int32),
                            t[keep].astype(np.int64), name="hubs")


@pytest.mark.parametrize("cls", PATH_CLASSES[:8] + WEDGE_CLASSES[:2] + WEDGE_CLASSES[4:6])
def test_batch_hub_windows(tcb, torch_mod, cls):
    """Windows of thousands of entries: the rank pass's galloping leaves the
    tile and its staged entries, and later queries of a thread are bracketed
    by the previous query's bound; ascending and unordered deltas."""
    g = _hub_graph()
    G, og = build_both(tcb, torch_mod, g)
    for deltas in ([10, 1000, 20000, 90000], [90000, 0, 20000, 3]):
        Ws = tcb.tc_path_weights_batch(G, deltas, cls=cls)
        for W, d in zip(Ws, deltas):
            ow = og.weights(d, cls=bytes(cls))
            A = W.arrays()
            for name in ("lo_in", "a", "lo_out", "b"):
                assert np.array_equal(_u32(A[name]), getattr(ow, name)), (cls, d, name)
            assert np.array_equal(_u64(A["S"]), ow.S)
            assert W.status() == ow.status
