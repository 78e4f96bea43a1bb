"""Pins of the oracle's general anchor classes (section III: the sixteen
classes <alpha_1, alpha_3, beta_1, beta_3> of delta-centred 3-paths, the
remark after Claim "count" that their weight is d^alpha_u * d^alpha'_v over
the class's intervals, and the wedges of the 3-vertex case), of its anchor
choice (Algorithm Estimate: an anchor holding the earliest motif edge) and
of the exhaustive mode (proof of Claim "est": sum over anchors of CheckMotif
is the number of matches).  Everything is checked against literal
enumeration from the definitions (oracle/brute.py) on micro graphs."""
import itertools
import math

import numpy as np
import pytest

import oracle
import synthgraph as sg
from oracle import brute

CLASSES_3PATH = [bytes([m1, a1, m3, a3]) for m1 in (1, 2) for a1 in (0, 1)
                 for m3 in (1, 2) for a3 in (0, 1)]
CLASSES_WEDGE = [bytes([m1, a1, 0, 0]) for m1 in (1, 2) for a1 in (0, 1)] + \
                [bytes([0, 0, m3, a3]) for m3 in (1, 2) for a3 in (0, 1)]
# the wedge anchors a motif can have: the base edge is the earliest, so the
# other edge comes after it
CLASSES_WEDGE_ANCHORED = [c for c in CLASSES_WEDGE if c[1] == 1 or c[3] == 1]


def _mb(edges, nv):
    return sg.motif_bytes(edges, nv)


def random_motif(rng, nv):
    """A random connected motif on nv vertices (2..6 edges, parallel and
    antiparallel edges allowed) that has an anchor."""
    while True:
        ne = int(rng.integers(nv - 1, 7))
        edges = []
        for _ in range(ne):
            a, b = rng.choice(nv, size=2, replace=False)
            edges.append((int(a), int(b)))
        if oracle.anchor(_mb(edges, nv)) is not None:
            return edges


@pytest.mark.parametrize("cls", CLASSES_3PATH + CLASSES_WEDGE)
@pytest.mark.parametrize("seed", range(3))
def test_class_weight_total_equals_path_enumeration(cls, seed):
    """Sum of w_e = number of delta-centred paths of the class (closed
    windows), for all 16 path classes and the 8 wedge classes."""
    g = sg.gen_micro(100 + seed, n=5, m=20, t_span=10)
    og = oracle.OracleGraph.from_graph(g)
    for delta in (0, 2, 6):
        w = og.weights(delta, cls=cls)
        assert w.status == 0
        assert w.W == len(brute.enumerate_class_paths(g.src, g.dst, g.t, delta, cls))


@pytest.mark.parametrize("cls", CLASSES_3PATH + CLASSES_WEDGE_ANCHORED)
def test_enumeration_visits_every_class_path_once(cls):
    """The exhaustive mode's ranks 0..W-1 map one to one onto the class's
    paths (the integer CDF, then j = j1 * b + j3)."""
    g = sg.gen_micro(7, n=5, m=18, t_span=8)
    og = oracle.OracleGraph.from_graph(g)
    w = og.weights(5, cls=cls)
    # any motif of this class serves to drive the enumeration
    mb = _class_motif(cls)
    E = og.enumerate(w, [mb], per_sample=True)
    got = sorted(zip(E.e1.tolist(), E.e2.tolist(), E.e3.tolist()))
    want = sorted(brute.enumerate_class_paths(g.src, g.dst, g.t, 5, cls))
    assert got == want


def _class_motif(cls):
    """A motif whose anchor has class cls: centre (1 -> 2) of rank r_c, the
    side edges placed before or after it as the class says."""
    m1, a1, m3, a3 = cls
    centre = (1, 2)
    parts = []  # (rank key, edge)
    if m1:
        parts.append((1 if a1 else -1, (0, 1) if m1 == 1 else (1, 0)))
    if m3:
        parts.append((2 if a3 else -2, (3, 2) if m3 == 1 else (2, 3)))
    parts.append((0, centre))
    edges = [e for _, e in sorted(parts)]
    if m1 and m3:
        nv = 4
    else:
        # 3 vertices: relabel {1, 2, other} to {0, 1, 2}
        nv = 3
        vs = sorted({x for e in edges for x in e})
        ren = {v: i for i, v in enumerate(vs)}
        edges = [(ren[a], ren[b]) for a, b in edges]
    mb = _mb(edges, nv)
    an = oracle.anchor(mb)
    assert an is not None and an[0] == cls, (cls, edges, an)
    return mb


def _open(cls, side1, side3):
    c = bytearray(cls)
    if side1 and c[0]:
        c[1] |= oracle.WINDOW_OPEN
    if side3 and c[2]:
        c[3] |= oracle.WINDOW_OPEN
    return bytes(c)


@pytest.mark.parametrize("cls", CLASSES_3PATH + CLASSES_WEDGE)
@pytest.mark.parametrize("opens", [(1, 0), (0, 1), (1, 1)])
def test_open_window_weight_total_equals_path_enumeration(cls, opens):
    """Windows open at the centre time ([t - delta, t) or (t, t + delta]):
    sum of w_e = number of class paths whose side times differ from the
    centre's, on micro graphs full of equal times; never above the closed
    total."""
    oc = _open(cls, *opens)
    for seed in range(3):
        g = sg.gen_micro(300 + seed, n=5, m=22, t_span=6)
        og = oracle.OracleGraph.from_graph(g)
        for delta in (0, 2, 5):
            w = og.weights(delta, cls=oc)
            assert w.status == 0
            assert w.W == len(brute.enumerate_class_paths(g.src, g.dst, g.t, delta, oc))
            assert w.W <= og.weights(delta, cls=cls).W


@pytest.mark.parametrize("cls", CLASSES_3PATH + CLASSES_WEDGE_ANCHORED)
def test_open_window_enumeration_visits_every_path_once(cls):
    oc = _open(cls, 1, 1)
    g = sg.gen_micro(17, n=5, m=18, t_span=6)
    og = oracle.OracleGraph.from_graph(g)
    w = og.weights(4, cls=oc)
    E = og.enumerate(w, [_class_motif(cls)], per_sample=True)
    got = sorted(zip(E.e1.tolist(), E.e2.tolist(), E.e3.tolist()))
    assert got == sorted(brute.enumerate_class_paths(g.src, g.dst, g.t, 4, oc))


@pytest.mark.parametrize("nv", [3, 4])
@pytest.mark.parametrize("seed", range(6))
def test_open_windows_keep_every_match(nv, seed):
    """A match's times increase strictly, so its anchor's side times differ
    from the centre's: the windows open at the centre time still give the
    exact count C over all anchors, with W no larger."""
    rng = np.random.default_rng(5000 + 100 * nv + seed)
    M = random_motif(rng, nv)
    mb = _mb(M, nv)
    cls = oracle.anchor(mb)[0]
    oc = _open(cls, 1, 1)
    g = sg.gen_micro_planted(50 + seed, M, copies=3, n=6, noise=8, t_span=12)
    og = oracle.OracleGraph.from_graph(g)
    for delta in (3, 8, 30):
        C = brute.count_matches(g.src, g.dst, g.t, M, delta)
        w = og.weights(delta, cls=oc)
        E = og.enumerate(w, [mb])
        assert E.status == 0 and E.cnt[0] == C, (M, delta, E.cnt, C)
        assert w.W <= og.weights(delta, cls=cls).W


def test_open_window_bytes_checked():
    """Only bits 0 and 1 of an `after` byte have a meaning."""
    g = sg.gen_micro(3, n=5, m=10, t_span=6)
    og = oracle.OracleGraph.from_graph(g)
    assert og.weights(3, cls=bytes([1, 4, 2, 1])).status == oracle.OR_ARG
    assert og.weights(3, cls=bytes([1, 2, 2, 3])).status == 0


@pytest.mark.parametrize("nv", [3, 4])
@pytest.mark.parametrize("seed", range(12))
def test_sum_checkmotif_over_anchors_equals_match_count(nv, seed):
    """Proof of Claim "est" for general anchors: every match has exactly one
    anchor, so the sum of CheckMotif over all anchors of the motif's class is
    C, counted here by literal enumeration of edge combinations."""
    rng = np.random.default_rng(1000 * nv + seed)
    M = random_motif(rng, nv)
    mb = _mb(M, nv)
    cls = oracle.anchor(mb)[0]
    g = sg.gen_micro_planted(seed, M, copies=3, n=6, noise=6)
    og = oracle.OracleGraph.from_graph(g)
    for delta in (3, 8, 30):
        C = brute.count_matches(g.src, g.dst, g.t, M, delta)
        assert og.brute_count(mb, delta) == C
        w = og.weights(delta, cls=cls)
        E = og.enumerate(w, [mb])
        assert E.status == 0 and E.cnt[0] == C, (M, delta, E.cnt, C)
        st, sx, _, nz = og.exhaustive(w, mb)
        assert st == 0 and sx == C and nz == int(E.hits[0])


def test_planted_random_motifs_have_matches():
    total = 0
    for nv in (3, 4):
        for seed in range(12):
            rng = np.random.default_rng(1000 * nv + seed)
            M = random_motif(rng, nv)
            g = sg.gen_micro_planted(seed, M, copies=3, n=6, noise=6)
            total += brute.count_matches(g.src, g.dst, g.t, M, 30) > 0
    assert total >= 18


def test_anchor_choice_examples():
    # the spine: ranks 0, 1, 2 form A -> B -> C -> D
    assert oracle.anchor(_mb(sg.MOTIFS["M4-0"], 4)) == (bytes([1, 0, 2, 1]), 3, [0, 1, 2],
                                                        [0, 1, 2])
    # A -> B (0), C -> D (1), B -> C (2), D -> A (3): the path A-B-C-D with
    # centre B -> C of rank 2, both sides before it
    a = oracle.anchor(_mb([(0, 1), (2, 3), (1, 2), (3, 0)], 4))
    assert a == (bytes([1, 0, 2, 0]), 3, [0, 2, 1], [0, 2, 1])
    # a wedge: base A -> B (0) and A -> C (1) after it from A's out-list
    # (the <+,>> wedge of the 3-vertex description), closed by C -> B
    a = oracle.anchor(_mb([(0, 1), (0, 2), (2, 1)], 3))
    assert a == (bytes([2, 1, 0, 0]), 2, [1, 0], [1, 0, -1])
    # B -> C (0) then A -> B (1): the side edge is an in-edge of the base's
    # source, after it
    a = oracle.anchor(_mb([(1, 2), (0, 1), (2, 0)], 3))
    assert a[0] == bytes([1, 1, 0, 0]) and a[1] == 2
    # no anchor: a 3-star, and a motif over two vertices
    assert oracle.anchor(_mb([(0, 1), (0, 2), (0, 3)], 4)) is None
    assert oracle.anchor(_mb([(0, 1), (1, 0)], 3)) is None


def test_b_statistics_by_grouping_matches():
    """The exhaustive mode's hits, xmax and m2 are the count of anchors with
    a match, the largest number of matches on one anchor and the sum of
    squares (the B statistics): checked against per-anchor CheckMotif
    values gathered one by one."""
    M = sg.MOTIFS["S5-paw"]
    mb = _mb(M, 4)
    g = sg.gen_micro_planted(4, M, copies=4, n=6, noise=8)
    og = oracle.OracleGraph.from_graph(g)
    w = og.weights(30)
    E = og.enumerate(w, [mb], per_sample=True)
    xs = []
    for e1, e2, e3 in zip(E.e1.tolist(), E.e2.tolist(), E.e3.tolist()):
        st, X = og.check_motif(mb, 30, e1, e2, e3)
        xs.append(X)
    xs = np.array(xs, dtype=np.float64)
    assert E.cnt[0] == int(xs.sum()) and int(E.hits[0]) == int((xs > 0).sum())
    assert int(E.xmax[0]) == int(xs.max()) and E.m2[0] == pytest.approx(float((xs ** 2).sum()))
    assert np.array_equal(E.X[0], xs.astype(np.uint64))


@pytest.mark.parametrize("cls_motif", [
    ([(0, 1), (2, 3), (1, 2), (3, 0)], 4),      # centre of rank 2, both sides before
    ([(1, 2), (2, 3), (1, 0), (3, 0)], 4),      # centre of rank 0, both sides after
    ([(0, 1), (0, 2), (2, 1)], 3),              # the <+,>> wedge
    ([(1, 2), (0, 1), (2, 0), (0, 1)], 3),      # in-edge after the base, a repeated pair
])
def test_general_class_estimator_unbiased_over_seeds(cls_motif):
    """E[C_hat] = C for anchors of other classes: the mean of 64 estimates
    lies within 4.5 standard errors of the exact count, with the exact
    per-sample variance from enumeration (Var = W * sum X^2 - C^2)."""
    M, nv = cls_motif
    mb = _mb(M, nv)
    cls = oracle.anchor(mb)[0]
    g = sg.gen_micro_planted(11, M, copies=6, n=7, noise=10, t_span=30)
    og = oracle.OracleGraph.from_graph(g)
    delta = 12
    w = og.weights(delta, cls=cls)
    st, C, sx2, _ = og.exhaustive(w, mb)
    assert st == 0 and C > 0 and C == brute.count_matches(g.src, g.dst, g.t, M, delta)
    W, k, seeds = w.W, 2000, 64
    var1 = W * sx2 - C * C            # variance of one sample's W * X
    ests = [og.sample(w, [mb], k, s, 9).est[0] for s in range(1, seeds + 1)]
    se = math.sqrt(var1 / k / seeds)
    assert abs(np.mean(ests) - C) <= 4.5 * se + 1e-9, (np.mean(ests), C, se)


def test_mixed_classes_in_one_call_rejected():
    g = sg.gen_micro(3, n=5, m=12, t_span=8)
    og = oracle.OracleGraph.from_graph(g)
    w = og.weights(5)
    other = _mb([(0, 1), (2, 3), (1, 2), (3, 0)], 4)   # another class
    E = og.sample(w, [sg.motif_bytes(sg.MOTIFS["M4-0"]), other], 10, 1)
    assert E.status == oracle.OR_ARG


@pytest.mark.parametrize("motif", [
    ([(0, 1), (1, 2), (2, 3)], 4),                 # the anchor alone: a temporal 3-path
    ([(0, 1), (0, 2)], 3),                         # the anchor alone: a temporal wedge
    ([(1, 2), (2, 3), (1, 0)], 4),                 # centre first, both sides after it
    ([(0, 1), (2, 3), (3, 1), (1, 2)], 4),         # a list between two anchor edges
    ([(0, 1), (1, 2), (0, 2), (0, 2)], 3),         # a wedge closed twice
])
@pytest.mark.parametrize("seed", range(3))
def test_fixed_motifs_on_dense_micro_graphs(motif, seed):
    """Dense random micro graphs (many anchors whose span exceeds delta):
    sum over anchors of CheckMotif = literal match count, for delta from 0
    up to past the time span."""
    M, nv = motif
    mb = _mb(M, nv)
    cls = oracle.anchor(mb)[0]
    g = sg.gen_micro(500 + seed, n=5, m=18, t_span=12)
    og = oracle.OracleGraph.from_graph(g)
    for delta in (0, 1, 2, 4, 7, 13):
        C = brute.count_matches(g.src, g.dst, g.t, M, delta)
        w = og.weights(delta, cls=cls)
        E = og.enumerate(w, [mb])
        assert E.status == 0 and E.cnt[0] == C, (M, delta, E.cnt[0], C)
