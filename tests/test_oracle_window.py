"""Pins of the oracle's window proposal (not part of the paper; an extension
of the importance-sampling estimator): the centre edge is drawn with
probability h_p G1_p G3_p / Q and each side's edge with probability g / G
over its window's factors, so a path has probability h_p g1 g3 / Q and the
per-sample value X Q / (h_p g1 g3) stays unbiased (Claim "est" for the
importance-weighted draw).  Checked against direct computation, exact
rational expectation over every path, the literal match count, bit-exact
reduction to the plain and the centre-only estimators, a chi-square test of
the pick distribution and a z-test over seeds with the exact variance."""
import math
from fractions import Fraction

import numpy as np
import pytest

import oracle
import synthgraph as sg
from oracle import learn

M40 = sg.motif_bytes(sg.MOTIFS["M4-0"])
SIX = [sg.motif_bytes(sg.MOTIFS[x]) for x in sg.SIX_MOTIFS]


def _factor(d, quarter, cap):
    r2 = math.isqrt(1 + d)
    r4 = math.isqrt(r2)
    f = [1, r4, r2, r2 * r4, r2 * r2][quarter]
    return min(f, cap)


@pytest.mark.parametrize("quarter,cap", [(0, 1), (1, 7), (2, 65535), (3, 40), (4, 9)])
def test_window_factors_by_direct_computation(quarter, cap):
    g = sg.gen_micro(3, n=9, m=60, t_span=30)
    og = oracle.OracleGraph.from_graph(g)
    f_in, f_out = og.window_factors(quarter, cap)
    o = og.orders()
    deg = np.bincount(g.src, minlength=g.n) + np.bincount(g.dst, minlength=g.n)
    want_in = [_factor(int(deg[g.src[e]]), quarter, cap) for e in o["in_eid"]]
    want_out = [_factor(int(deg[g.dst[e]]), quarter, cap) for e in o["out_eid"]]
    assert list(f_in) == want_in and list(f_out) == want_out


def test_factor_integer_roots_at_large_degrees():
    # isqrt exactness where a float square root rounds up
    for d in [0, 1, 2, 3, 15, 16, 24, 99, 2**26 - 2, 2**26 - 1, 2**31 - 2, 2**31 + 7]:
        r2 = math.isqrt(1 + d)
        assert _factor(d, 2, 65535) == min(r2, 65535)
        assert _factor(d, 1, 65535) == min(math.isqrt(r2), 65535)


@pytest.mark.parametrize("cls", [(1, 0, 2, 1), (2, 1, 1, 0), (1, 1, 0, 0), (0, 0, 2, 0)])
def test_window_q_scan_by_direct_computation(cls):
    g = sg.gen_micro(5, n=8, m=70, t_span=25)
    og = oracle.OracleGraph.from_graph(g)
    w = og.weights(9, cls=bytes(cls))
    f_in, f_out = og.window_factors(2, 5)
    rng = np.random.default_rng(1)
    h = rng.integers(1, 9, size=og.m).astype(np.uint32)
    wq = og.proposal_window(w, h, f_in, f_out)
    assert wq.status == 0
    ps_in = np.concatenate([[0], np.cumsum(f_in.astype(np.int64))])
    ps_out = np.concatenate([[0], np.cumsum(f_out.astype(np.int64))])
    side = {1: ps_in, 2: ps_out}
    run = 0
    for p in range(og.m):
        assert int(wq.S[p]) == run
        G1 = 1 if cls[0] == 0 else int(side[cls[0]][w.lo_in[p] + w.a[p]] - side[cls[0]][w.lo_in[p]])
        G3 = 1 if cls[2] == 0 else int(side[cls[2]][w.lo_out[p] + w.b[p]] -
                                       side[cls[2]][w.lo_out[p]])
        run += int(h[p]) * G1 * G3
    assert int(wq.S[og.m]) == run
    if cls[0]:
        assert np.array_equal(wq.ps1, side[cls[0]].astype(np.uint64))
    if cls[2]:
        assert np.array_equal(wq.ps3, side[cls[2]].astype(np.uint64))


def test_window_q_overflow_flagged():
    g, _ = sg.gen_gadget(40, 40, 1)
    og = oracle.OracleGraph.from_graph(g)
    w = og.weights(10**6)
    big = np.full(og.m, 2**31, np.uint32)
    assert og.proposal_window(w, None, big, big).status & 2  # window sums beyond 2^32


def test_unit_factors_reduce_to_plain_and_centre_only_bit_exactly():
    g = sg.gen_tiny()
    og = oracle.OracleGraph.from_graph(g)
    for delta in (3600, 20000):
        w = og.weights(delta)
        ones = np.ones(og.m, np.uint32)
        wq = og.proposal_window(w, None, ones, ones)
        assert wq.W == w.W
        P = og.sample(w, SIX, 20000, 5, per_sample=True)
        Q = og.sample(wq, SIX, 20000, 5, per_sample=True)
        assert P.status == Q.status == 0
        for f in ("e1", "e2", "e3", "X", "P"):
            assert np.array_equal(getattr(P, f), getattr(Q, f)), f
        assert Q.cnt == [c << 64 for c in P.cnt]
        assert np.array_equal(P.est.view(np.uint64), Q.est.view(np.uint64))
        # with a centre factor h: the same as the centre-only proposal
        s = learn.quant_shift(w.W)
        h = np.random.default_rng(delta).integers(1, 2**s + 1, size=og.m).astype(np.uint32)
        H = og.sample(og.proposal(w, h), SIX, 20000, 6, per_sample=True)
        HW = og.sample(og.proposal_window(w, h, ones, ones), SIX, 20000, 6, per_sample=True)
        for f in ("e1", "e2", "e3", "X", "P"):
            assert np.array_equal(getattr(H, f), getattr(HW, f)), f
        assert H.cnt == HW.cnt and np.array_equal(H.est.view(np.uint64), HW.est.view(np.uint64))


def _paths(og, w, wq, f_in, f_out, h, motif):
    """Every path with its proposal probability h g1 g3 / Q and X."""
    o = og.orders()
    side_f = {1: f_in, 2: f_out}
    cls = w.cls
    out = []
    for p in range(og.m):
        hp = 1 if h is None else int(h[p])
        r1 = range(int(w.a[p]))
        r3 = range(int(w.b[p]))
        for j1 in r1:
            for j3 in r3:
                e1 = -1 if cls[0] == 0 else int((o["in_eid"] if cls[0] == 1 else o["out_eid"])
                                                [w.lo_in[p] + j1])
                e3 = -1 if cls[2] == 0 else int((o["in_eid"] if cls[2] == 1 else o["out_eid"])
                                                [w.lo_out[p] + j3])
                g1 = 1 if cls[0] == 0 else int(side_f[cls[0]][w.lo_in[p] + j1])
                g3 = 1 if cls[2] == 0 else int(side_f[cls[2]][w.lo_out[p] + j3])
                _, X = og.check_motif(motif, w.delta, e1, int(o["out_eid"][p]), e3)
                out.append((p, j1, j3, hp * g1 * g3, X))
    return out


@pytest.mark.parametrize("seed", range(4))
def test_window_exact_expectation_equals_count(seed):
    M = sg.MOTIFS[sg.SIX_MOTIFS[seed % 6]]
    g = sg.gen_micro_planted(seed, M, copies=3, n=7, noise=10)
    og = oracle.OracleGraph.from_graph(g)
    mb = sg.motif_bytes(M)
    rng = np.random.default_rng(seed)
    for delta in (4, 9, 40):
        w = og.weights(delta)
        f_in = rng.integers(1, 30, size=og.m).astype(np.uint32)
        f_out = rng.integers(1, 30, size=og.m).astype(np.uint32)
        h = rng.integers(1, 5, size=og.m).astype(np.uint32)
        wq = og.proposal_window(w, h, f_in, f_out)
        Q = wq.W
        paths = _paths(og, w, wq, f_in, f_out, h, mb)
        # the proposal probabilities sum to one
        assert sum(Fraction(q, Q) for *_, q, _ in paths) == 1
        E = sum(Fraction(q, Q) * Fraction((X << 64) // q, 1 << 64) * Q for *_, q, X in paths if X)
        C = sum(X for *_, X in paths)
        assert C == og.brute_count(mb, delta)
        assert abs(E - C) <= 1
        # factors that are powers of two: the correction is exact
        f2 = (1 << rng.integers(0, 5, size=og.m)).astype(np.uint32)
        wq2 = og.proposal_window(w, None, f2, f2)
        p2 = _paths(og, w, wq2, f2, f2, None, mb)
        E2 = sum(Fraction(q, wq2.W) * Fraction((X << 64) // q, 1 << 64) * wq2.W
                 for *_, q, X in p2 if X)
        assert E2 == C


def test_window_pick_distribution_chi_square():
    """Paths drawn by the window proposal follow h g1 g3 / Q."""
    g = sg.gen_micro(11, n=6, m=30, t_span=14)
    og = oracle.OracleGraph.from_graph(g)
    w = og.weights(6)
    rng = np.random.default_rng(4)
    f_in = rng.integers(1, 6, size=og.m).astype(np.uint32)
    f_out = rng.integers(1, 6, size=og.m).astype(np.uint32)
    h = rng.integers(1, 4, size=og.m).astype(np.uint32)
    wq = og.proposal_window(w, h, f_in, f_out)
    paths = _paths(og, w, wq, f_in, f_out, h, M40)
    assert 20 <= len(paths) <= 400
    k = 400000
    E = og.sample(wq, [M40], k, 9, per_sample=True)
    o = og.orders()
    pos_in = {int(e): i for i, e in enumerate(o["in_eid"])}
    pos_out = {int(e): i for i, e in enumerate(o["out_eid"])}
    seen = {}
    for p, e1, e3 in zip(E.P, E.e1, E.e3):
        key = (int(p), pos_in[int(e1)] - int(w.lo_in[p]), pos_out[int(e3)] - int(w.lo_out[p]))
        seen[key] = seen.get(key, 0) + 1
    chi2 = 0.0
    for p, j1, j3, q, _ in paths:
        exp = k * q / wq.W
        chi2 += (seen.get((p, j1, j3), 0) - exp) ** 2 / exp
    assert sum(seen.values()) == k and set(seen) <= {(p, j1, j3) for p, j1, j3, *_ in paths}
    dof = len(paths) - 1
    assert chi2 < dof + 6 * math.sqrt(2 * dof), (chi2, dof)


def test_window_unbiased_over_seeds_with_exact_variance():
    g = sg.gen_micro_planted(2, sg.MOTIFS["M4-0"], copies=4, n=8, noise=14)
    og = oracle.OracleGraph.from_graph(g)
    w = og.weights(12)
    f_in, f_out = og.window_factors(2, 65535)
    wq = og.proposal_window(w, None, f_in, f_out)
    paths = _paths(og, w, wq, f_in, f_out, None, M40)
    C = sum(X for *_, X in paths)
    Q = wq.W
    var_w = sum(Fraction(X * X, q) for *_, q, X in paths) * Q - C * C
    assert C > 0
    k, R = 4000, 40
    ests = np.array([og.sample(wq, [M40], k, seed).est[0] for seed in range(1, R + 1)])
    z = (ests.mean() - C) / math.sqrt(max(float(var_w), 1e-9) / k / R)
    assert abs(z) < 4.5, z
