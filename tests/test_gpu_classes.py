"""GPU parity for the general anchor classes (section III: the classes
<alpha_1, alpha_3, beta_1, beta_3> of delta-centred 3-paths and the wedges
of the 3-vertex case; Algorithm Estimate's anchor holding the earliest
edge) and for the exhaustive mode (proof of Claim "est": the sum over all
anchors of CheckMotif is the exact count).  Everything through the C ABI
against the oracle on the same seeded inputs: windows and S bit for bit for
every class, per-sample anchors and counts bit for bit, exhaustive counts
against literal match enumeration."""
import numpy as np
import pytest

import oracle
import synthgraph as sg
from oracle import brute
from test_gpu_parity import _u32, _u64, build_both

pytestmark = pytest.mark.gpu

PATH_CLASSES = [(m1, a1, m3, a3) for m1 in (1, 2) for a1 in (0, 1) for m3 in (1, 2)
                for a3 in (0, 1)]
WEDGE_CLASSES = [(m1, a1, 0, 0) for m1 in (1, 2) for a1 in (0, 1)] + \
                [(0, 0, m3, a3) for m3 in (1, 2) for a3 in (0, 1)]

# motifs of several classes: (edges, nv)
MOTIFS = [
    ([(0, 1), (2, 3), (1, 2), (3, 0)], 4),              # centre of rank 2, both sides before
    ([(1, 2), (2, 3), (1, 0), (3, 0)], 4),              # centre first, both sides after
    ([(0, 1), (1, 2), (2, 3), (0, 2), (3, 1)], 4),      # the spine with two chords
    ([(2, 1), (1, 0), (2, 3), (3, 1), (0, 3)], 4),      # out-edge at u before the centre
    ([(0, 1), (0, 2), (2, 1)], 3),                      # the <+,>> wedge, closed
    ([(1, 2), (0, 1), (2, 0), (0, 1)], 3),              # in-edge after the base, repeated pair
    ([(0, 1), (2, 1), (0, 2), (2, 0), (1, 0)], 3),      # wedge at v, five edges
    ([(0, 1), (1, 2), (2, 3)], 4),                      # the anchor alone
    ([(0, 1), (0, 2)], 3),                              # the wedge alone
]


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


def _weights_equal(Wt, ow):
    A = Wt.arrays()
    for name in ("lo_in", "a", "lo_out", "b"):
        assert np.array_equal(_u32(A[name]), getattr(ow, name)), name
    assert np.array_equal(_u64(A["S"]), ow.S)
    assert Wt.status() == ow.status


def _sample_equal(tcb, G, Wt, og, ow, motifs, k, seed, stream=0, i0=0):
    mb = [sg.motif_bytes(M, nv) for M, nv in motifs]
    R = tcb.tc_sample_estimate(G, Wt, motifs, k, seed, stream, i0, per_sample=True)
    E = og.sample(ow, mb, k, seed, stream, i0, per_sample=True)
    st = int(R.status.item()) & 0xFFFFFFFF
    assert st == E.status
    assert np.array_equal(R.e1.cpu().numpy(), E.e1)
    assert np.array_equal(R.e2.cpu().numpy(), E.e2)
    assert np.array_equal(R.e3.cpu().numpy(), E.e3)
    assert np.array_equal(_u64(R.X), E.X)
    assert R.counts() == E.cnt
    assert np.array_equal(_u64(R.hits), E.hits)
    assert np.array_equal(_u64(R.xmax), E.xmax)
    assert np.array_equal(R.estimate.cpu().numpy().view(np.uint64), E.est.view(np.uint64))
    return R, E


@pytest.mark.parametrize("cls", PATH_CLASSES + WEDGE_CLASSES)
def test_class_weights(tcb, tiny, cls):
    g, G, og = tiny
    for delta in (0, 3600, 40000):
        Wt = tcb.tc_path_weights(G, delta, cls=cls)
        ow = og.weights(delta, cls=bytes(cls))
        _weights_equal(Wt, ow)
        assert Wt.c.cls.as_tuple() == cls


@pytest.mark.parametrize("mi", range(len(MOTIFS)))
def test_class_sampling_tiny(tcb, tiny, mi):
    g, G, og = tiny
    M, nv = MOTIFS[mi]
    cls, na, order = tcb.tc_motif_anchor(M, nv)
    assert oracle.anchor(sg.motif_bytes(M, nv))[0] == bytes(cls)
    for delta, seed in ((3600, 1), (40000, 2)):
        Wt = tcb.tc_path_weights(G, delta, cls=cls)
        ow = og.weights(delta, cls=bytes(cls))
        _sample_equal(tcb, G, Wt, og, ow, [(M, nv)], 60000, seed, 3, 5)


@pytest.mark.parametrize("nv", [3, 4])
@pytest.mark.parametrize("seed", range(6))
def test_random_motifs_planted(tcb, torch_mod, nv, seed):
    """Random motifs (the oracle's pins use the same recipe) on micro graphs
    where they are planted: per-sample parity, and the exhaustive count
    equals the literal match count."""
    rng = np.random.default_rng(1000 * nv + seed)
    while True:
        ne = int(rng.integers(nv - 1, 7))
        M = [tuple(int(x) for x in rng.choice(nv, size=2, replace=False)) for _ in range(ne)]
        if oracle.anchor(sg.motif_bytes(M, nv)) is not None:
            break
    cls = tcb.tc_motif_anchor(M, nv)[0]
    g = sg.gen_micro_planted(seed, M, copies=3, n=6, noise=6)
    G, og = build_both(tcb, torch_mod, g)
    for delta in (3, 8, 30):
        Wt = tcb.tc_path_weights(G, delta, cls=cls)
        ow = og.weights(delta, cls=bytes(cls))
        _weights_equal(Wt, ow)
        _sample_equal(tcb, G, Wt, og, ow, [(M, nv)], 5000, seed + 1)
        R = tcb.tc_exhaustive_count(G, Wt, [(M, nv)])
        R.check()
        assert R.counts()[0] == brute.count_matches(g.src, g.dst, g.t, M, delta)


def test_several_motifs_of_one_class_and_batch(tcb, tiny):
    """Motifs sharing class and rank order in one call, and the batched
    sequence over three deltas, equal the single calls and the oracle."""
    g, G, og = tiny
    base = [(0, 1), (2, 3), (1, 2)]            # centre of rank 2, sides before it
    motifs = [(base + [(3, 0)], 4), (base + [(3, 0), (0, 2)], 4), (base + [(1, 3), (3, 0)], 4),
              (base, 4)]
    cls = tcb.tc_motif_anchor(*motifs[0])[0]
    deltas = [600, 3600, 40000]
    Ws = [tcb.tc_path_weights(G, d, cls=cls) for d in deltas]
    outs = tcb.tc_batch_estimate(G, Ws, motifs, 40000, 9, 2, 0, per_sample=True)
    for d, W, o in zip(deltas, Ws, outs):
        s = tcb.tc_sample_estimate(G, W, motifs, 40000, 9, 2, 0, per_sample=True)
        assert o.counts() == s.counts()
        assert np.array_equal(_u64(o.X), _u64(s.X))
        ow = og.weights(d, cls=bytes(cls))
        E = og.sample(ow, [sg.motif_bytes(M, nv) for M, nv in motifs], 40000, 9, 2, 0)
        assert o.counts() == E.cnt


def test_mixed_anchors_rejected(tcb, tiny):
    g, G, og = tiny
    W = tcb.tc_path_weights(G, 3600)
    with pytest.raises(tcb.TCError) as e:
        tcb.tc_sample_estimate(G, W, [sg.MOTIFS["M4-0"], [(0, 1), (2, 3), (1, 2), (3, 0)]], 10, 1)
    assert e.value.code == tcb.TC_E_ARG
    # weights of another class
    with pytest.raises(tcb.TCError) as e:
        tcb.tc_sample_estimate(G, W, [[(0, 1), (0, 2), (2, 1)]], 10, 1)
    assert e.value.code == tcb.TC_E_ARG


@pytest.mark.parametrize("mi", [0, 2, 4, 6])
def test_exhaustive_per_rank_parity(tcb, torch_mod, mi):
    """Exhaustive mode, every rank: the anchor and X of each rank equal the
    oracle's enumeration; cnt, hits, xmax and m2 equal its totals; partial
    ranges add up and ranks past W contribute nothing."""
    M, nv = MOTIFS[mi]
    cls = tcb.tc_motif_anchor(M, nv)[0]
    g = sg.gen_micro_planted(mi, M, copies=5, n=7, noise=20, t_span=40)
    G, og = build_both(tcb, torch_mod, g)
    delta = 15
    Wt = tcb.tc_path_weights(G, delta, cls=cls)
    ow = og.weights(delta, cls=bytes(cls))
    Wn = ow.W
    assert Wn > 0
    R = tcb.tc_exhaustive_count(G, Wt, [(M, nv)], per_sample=True)
    E = og.enumerate(ow, [sg.motif_bytes(M, nv)], per_sample=True)
    R.check()
    assert np.array_equal(R.e1.cpu().numpy(), E.e1)
    assert np.array_equal(R.e2.cpu().numpy(), E.e2)
    assert np.array_equal(R.e3.cpu().numpy(), E.e3)
    assert np.array_equal(_u64(R.X), E.X)
    assert R.counts() == E.cnt and int(R.hits[0].item()) == int(E.hits[0])
    assert int(R.xmax[0].item()) == int(E.xmax[0])
    assert R.m2[0].item() == pytest.approx(E.m2[0], rel=1e-12)
    assert R.estimate[0].item() == float(E.cnt[0])
    assert E.cnt[0] == brute.count_matches(g.src, g.dst, g.t, M, delta)
    # ranges: [0, h), [h, W + 7) add up; the ranks past W give nothing
    h = Wn // 2
    a = tcb.tc_exhaustive_count(G, Wt, [(M, nv)], 0, h)
    b = tcb.tc_exhaustive_count(G, Wt, [(M, nv)], h, Wn - h + 7)
    assert a.counts()[0] + b.counts()[0] == E.cnt[0]


def test_exhaustive_tiny_six_motifs_and_b_statistics(tcb, tiny):
    """The exact count of the six motifs on the tiny workload (W ~ 4*10^5
    anchors) equals the oracle's enumeration and its backtracking count;
    hits, xmax and m2 give the B statistics of the experiments section."""
    g, G, og = tiny
    six = [sg.MOTIFS[n] for n in sg.SIX_MOTIFS]
    for delta in (3600, 20000):
        Wt = tcb.tc_path_weights(G, delta)
        ow = og.weights(delta)
        R = tcb.tc_exhaustive_count(G, Wt, six)
        R.check()
        E = og.enumerate(ow, [sg.motif_bytes(M) for M in six])
        assert R.counts() == E.cnt
        assert np.array_equal(_u64(R.hits), E.hits)
        assert np.array_equal(_u64(R.xmax), E.xmax)
        for j, M in enumerate(six):
            assert E.cnt[j] == og.brute_count(sg.motif_bytes(M), delta)
            assert R.m2[j].item() == pytest.approx(E.m2[j], rel=1e-12)


# ---- windows open at the centre time (TC_WINDOW_OPEN) ----------------------
def _open(cls, side1=True, side3=True):
    c = list(cls)
    if side1 and c[0]:
        c[1] |= 2
    if side3 and c[2]:
        c[3] |= 2
    return tuple(c)


@pytest.fixture(scope="module")
def ties(tcb, torch_mod):
    """A micro graph full of equal times (300 edges over 21 time values)."""
    g = sg.gen_micro(400, n=6, m=300, t_span=20)
    G, og = build_both(tcb, torch_mod, g)
    return g, G, og


@pytest.mark.parametrize("cls", PATH_CLASSES + WEDGE_CLASSES)
def test_open_window_weights(tcb, tiny, ties, cls):
    """Every class with one or both windows open at the centre time: windows
    and S equal the oracle's on the tiny graph and on a graph of ties, and W
    is never above the closed windows' W."""
    for opens in ((1, 0), (0, 1), (1, 1)):
        oc = _open(cls, *opens)
        for g, G, og in (tiny, ties):
            for delta in (0, 5, 3600, 40000):
                Wt = tcb.tc_path_weights(G, delta, cls=oc)
                _weights_equal(Wt, og.weights(delta, cls=bytes(oc)))
                assert Wt.total() <= tcb.tc_path_weights(G, delta, cls=cls).total()


def test_open_window_batch_hubs_and_sampling(tcb, torch_mod):
    """Open windows through the batched rank passes on hub windows of
    thousands of entries (galloping past the tile, bracketing by the previous
    query), then per-sample sampling parity on them."""
    from test_gpu_weights_batch import _hub_graph
    g = _hub_graph()
    G, og = build_both(tcb, torch_mod, g)
    oc = (1, 2, 2, 3)
    deltas = [10, 1000, 20000, 90000]
    Ws = tcb.tc_path_weights_batch(G, deltas, cls=oc)
    for W, d in zip(Ws, deltas):
        _weights_equal(W, og.weights(d, cls=bytes(oc)))
    M40 = (sg.MOTIFS["M4-0"], 4)
    _sample_equal(tcb, G, Ws[2], og, og.weights(20000, cls=bytes(oc)), [M40], 20000, 3)


@pytest.mark.parametrize("nv", [3, 4])
@pytest.mark.parametrize("seed", range(3))
def test_open_windows_exhaustive_equals_count(tcb, torch_mod, nv, seed):
    """A match's times increase strictly, so the open windows keep every
    anchor: the exhaustive count over them is the literal match count."""
    rng = np.random.default_rng(7000 + 100 * nv + seed)
    while True:
        ne = int(rng.integers(nv - 1, 7))
        M = [tuple(int(x) for x in rng.choice(nv, size=2, replace=False)) for _ in range(ne)]
        if oracle.anchor(sg.motif_bytes(M, nv)) is not None:
            break
    oc = _open(tcb.tc_motif_anchor(M, nv)[0])
    g = sg.gen_micro_planted(60 + seed, M, copies=3, n=6, noise=8, t_span=12)
    G, og = build_both(tcb, torch_mod, g)
    for delta in (3, 8, 30):
        Wt = tcb.tc_path_weights(G, delta, cls=oc)
        _weights_equal(Wt, og.weights(delta, cls=bytes(oc)))
        R = tcb.tc_exhaustive_count(G, Wt, [(M, nv)])
        R.check()
        assert R.counts()[0] == brute.count_matches(g.src, g.dst, g.t, M, delta)
