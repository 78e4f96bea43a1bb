"""Pins for the CPU oracle: each test checks it against something other than
itself -- published known-answer vectors, the definition of a match
enumerated literally, closed forms, library sorts, exact uniformity of the
range reduction, and statistical properties the paper proves."""
import math
import os

import numpy as np
import pytest

import synthgraph as sg
import oracle
from oracle import brute

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
M40 = sg.motif_bytes(sg.MOTIFS["M4-0"])


# ---------------------------------------------------------------- RNG ------
def test_philox_known_answers():
    with open(os.path.join(GOLDEN, "philox4x32_10_kat.txt")) as f:
        rows = [l.split() for l in f if l.strip() and not l.startswith("#")]
    assert len(rows) == 3
    for r in rows:
        v = [int(x, 16) for x in r]
        assert oracle.philox4x32_10(v[0:4], v[4:6]) == v[6:10]


def _philox_py(ctr, key):
    """Philox4x32-10 from the description in Salmon et al. (SC 2011): ten
    rounds of two 32x32->64 products whose halves are mixed with the other
    two words and the round key; the key is bumped by the two Weyl constants
    between rounds."""
    M0, M1, W0, W1, MASK = 0xD2511F53, 0xCD9E8D57, 0x9E3779B9, 0xBB67AE85, 0xFFFFFFFF
    x0, x1, x2, x3 = ctr
    k0, k1 = key
    for rnd in range(10):
        if rnd:
            k0, k1 = (k0 + W0) & MASK, (k1 + W1) & MASK
        p0, p1 = M0 * x0, M1 * x2
        x0, x1, x2, x3 = ((p1 >> 32) ^ x1 ^ k0, p1 & MASK, (p0 >> 32) ^ x3 ^ k1, p0 & MASK)
    return [x0, x1, x2, x3]


def test_philox_matches_independent_bigint_version():
    rng = np.random.default_rng(5)
    for _ in range(300):
        ctr = [int(v) for v in rng.integers(0, 2**32, size=4)]
        key = [int(v) for v in rng.integers(0, 2**32, size=2)]
        assert oracle.philox4x32_10(ctr, key) == _philox_py(ctr, key)


@pytest.mark.parametrize("s", [3 * 2**30, 2**32 - 5, 2**31 + 1, 1000003, 2**20 + 7, 7])
def test_lemire32_every_output_has_equal_preimages(s):
    """Exact uniformity: each output y has exactly floor(2^32 / s) accepted
    draws.  Checked by brute force over the preimage interval of sampled y."""
    rng = np.random.default_rng(s)
    want = (1 << 32) // s
    ys = rng.integers(0, s, size=12 if s > 2**16 else 3)
    if s == 7:
        ys = [0, 3, 6]
    for y in ys:
        y = int(y)
        lo = -((-y << 32) // s)          # ceil(y * 2^32 / s)
        hi = -((-(y + 1) << 32) // s)    # ceil((y+1) * 2^32 / s)
        if hi - lo > 5000:
            continue
        acc = 0
        for x in range(lo, hi):
            out = oracle.lemire32(x, s)
            if out is not None:
                assert out == y
                acc += 1
        assert acc == want, (s, y, acc, want)
    # draws outside the preimage interval never map to y
    assert oracle.lemire32(0, s) in (0, None)
    assert oracle.lemire32(2**32 - 1, s) in (s - 1, None)


@pytest.mark.parametrize("s", [2**64 - 12345, 3 * 2**62, 2**63 + 1, 2**64 - 1, 5 * 2**61 + 3])
def test_lemire64_every_output_has_equal_preimages(s):
    rng = np.random.default_rng(7)
    want = (1 << 64) // s
    for _ in range(40):
        y = int(rng.integers(0, 2**62)) * 4 % s
        lo = -((-y << 64) // s)
        hi = -((-(y + 1) << 64) // s)
        acc = 0
        for x in range(lo, hi):
            out = oracle.lemire64(x, s)
            if out is not None:
                assert out == y
                acc += 1
        assert acc == want


def test_lemire_chi2_against_biased_multiply_shift():
    """For s = 3*2^30 the plain multiply-shift map gives one output in three
    twice the mass; with rejection the three residue classes are balanced."""
    s = 3 * 2**30
    rng = np.random.default_rng(11)
    xs = rng.integers(0, 2**32, size=30000, dtype=np.uint64)
    cnt = np.zeros(3)
    for x in xs:
        y = oracle.lemire32(int(x), s)
        if y is not None:
            cnt[y % 3] += 1
    e = cnt.sum() / 3
    chi2 = ((cnt - e) ** 2 / e).sum()
    assert chi2 < 20.0  # 2 dof; the unrejected map gives chi2 ~ 1000s


# ------------------------------------------------------- adjacency --------
@pytest.mark.parametrize("seed", [0, 1, 2])
def test_orders_match_library_lexsort(seed):
    g = sg.gen_micro(seed, n=7, m=400, t_span=15)
    og = oracle.OracleGraph.from_graph(g)
    o = og.orders()
    eid = np.arange(g.m)
    assert np.array_equal(o["out_eid"], np.lexsort((eid, g.t, g.src)))
    assert np.array_equal(o["in_eid"], np.lexsort((eid, g.t, g.dst)))
    assert np.array_equal(o["pair_eid"], np.lexsort((eid, g.t, g.dst, g.src)))
    assert np.array_equal(o["out_off"], np.concatenate([[0], np.cumsum(np.bincount(g.src, minlength=g.n))]))
    assert np.array_equal(o["in_off"], np.concatenate([[0], np.cumsum(np.bincount(g.dst, minlength=g.n))]))


def test_window_counts_by_linear_scan():
    g = sg.gen_micro(5, n=9, m=600, t_span=40)
    delta = 6
    og = oracle.OracleGraph.from_graph(g)
    o = og.orders()
    w = og.weights(delta)
    S = 0
    for p in range(g.m):
        e = o["out_eid"][p]
        u, v, t = g.src[e], g.dst[e], g.t[e]
        ins = (g.dst == u) & (g.t >= t - delta) & (g.t <= t)
        outs = (g.src == v) & (g.t >= t) & (g.t <= t + delta)
        assert w.a[p] == ins.sum() and w.b[p] == outs.sum()
        before_in = ((g.dst == u) & (g.t < t - delta)).sum()
        before_out = ((g.src == v) & (g.t < t)).sum()
        assert w.lo_in[p] == o["in_off"][u] + before_in
        assert w.lo_out[p] == o["out_off"][v] + before_out
        assert int(w.S[p]) == S
        S += int(ins.sum()) * int(outs.sum())
    assert int(w.S[-1]) == S and w.status == 0


@pytest.mark.parametrize("seed", range(8))
def test_total_weight_equals_path_enumeration(seed):
    """Claim "count": sum_e w_e is the number of delta-centred <-,+,<,>> paths."""
    g = sg.gen_micro(seed, n=5, m=22, t_span=10)
    og = oracle.OracleGraph.from_graph(g)
    for delta in (0, 2, 5, 11):
        w = og.weights(delta)
        assert w.W == len(brute.enumerate_paths(g.src, g.dst, g.t, delta))


# ------------------------------------------------- closure / counts -------
@pytest.mark.parametrize("name", sg.SIX_MOTIFS)
@pytest.mark.parametrize("seed", range(4))
def test_sum_checkmotif_over_paths_equals_match_count(name, seed):
    """Proof of Claim "est": every match has exactly one anchor path, so the
    sum of CheckMotif over all W paths is C.  C is enumerated literally."""
    M = sg.MOTIFS[name]
    mb = sg.motif_bytes(M)
    g = sg.gen_micro_planted(seed, M, copies=2, n=6, noise=0 if len(M) >= 8 else 6)
    og = oracle.OracleGraph.from_graph(g)
    for delta in (4, 9, 25):
        C = brute.count_matches(g.src, g.dst, g.t, M, delta)
        assert og.brute_count(mb, delta) == C
        w = og.weights(delta)
        st, sx, _, _ = og.exhaustive(w, mb)
        assert st == 0 and sx == C, (name, seed, delta, sx, C)


def test_planted_micro_graphs_have_matches():
    total = 0
    for name in sg.SIX_MOTIFS:
        M = sg.MOTIFS[name]
        for seed in range(4):
            g = sg.gen_micro_planted(seed, M, copies=2, n=6, noise=0 if len(M) >= 8 else 6)
            total += brute.count_matches(g.src, g.dst, g.t, M, 25)
    assert total > 20


def test_tiny_workload_exhaustive_equals_backtracking():
    g = sg.gen_tiny()
    og = oracle.OracleGraph.from_graph(g)
    for name in sg.SIX_MOTIFS:
        mb = sg.motif_bytes(sg.MOTIFS[name])
        for delta in (3600, 20000):
            w = og.weights(delta)
            st, sx, _, _ = og.exhaustive(w, mb)
            assert st == 0 and sx == og.brute_count(mb, delta)


def test_list_count_vs_product_enumeration():
    rng = np.random.default_rng(3)
    for _ in range(300):
        l = int(rng.integers(0, 5))
        lists = [sorted(rng.integers(0, 8, size=int(rng.integers(0, 6))).tolist()) for _ in range(l)]
        st, X = oracle.list_count(lists)
        assert st == 0 and X == brute.list_count_bruteforce(lists)


def test_list_count_blocks_closed_form_and_overflow():
    # lists occupying disjoint increasing time blocks: count = product of sizes
    sizes = [5, 3, 7, 2]
    lists, base = [], 0
    for s in sizes:
        lists.append(list(range(base, base + s)))
        base += s
    assert oracle.list_count(lists) == (0, math.prod(sizes))
    # beyond 2^64: counts are 128-bit (2048^6 = 2^66 chains, exactly)
    big = [list(range(r * 4096, r * 4096 + 2048)) for r in range(6)]
    assert oracle.list_count(big) == (0, 2048**6)
    ok = [list(range(r * 4096, r * 4096 + 2048)) for r in range(5)] + [list(range(6 * 4096, 6 * 4096 + 511))]
    st, X = oracle.list_count(ok)
    assert st == 0 and X == 2048**5 * 511
    # and interleaved lists whose chain count passes 2^64: a closed form --
    # L_r = {r, r + 13, r + 26, ...} (n entries each, 13 lists): a chain picks
    # one entry per list with strictly increasing times, i.e. block indices
    # b_1 <= b_2 <= ... <= b_13 in [0, n): C(n + 12, 13)
    n = 400
    inter = [[r + 13 * i for i in range(n)] for r in range(13)]
    st, X = oracle.list_count(inter)
    assert st == 0 and X == math.comb(n + 12, 13) and X > 2**64


def test_fig1_walkthrough_fragments():
    with open(os.path.join(GOLDEN, "fig1_walkthrough.txt")) as f:
        rows = [l for l in f if l.strip() and not l.startswith("#")]
    for row in rows:
        head, edges = row.split("|")
        case, delta, want = head.split()
        E = [tuple(int(x) for x in e.split(",")) for e in edges.split()]
        src = np.array([e[0] for e in E], np.int32)
        dst = np.array([e[1] for e in E], np.int32)
        t = np.array([e[2] for e in E], np.int64)
        og = oracle.OracleGraph(4, src, dst, t)
        assert og.brute_count(M40, int(delta)) == int(want), case
        assert brute.count_matches(src, dst, t, sg.MOTIFS["M4-0"], int(delta)) == int(want)
        w = og.weights(int(delta))
        assert og.exhaustive(w, M40)[1] == int(want), case


@pytest.mark.parametrize("p,q,r", [(1, 1, 1), (3, 4, 1), (5, 2, 3), (7, 9, 4)])
def test_gadget_closed_forms(p, q, r):
    g, delta = sg.gen_gadget(p, q, r)
    og = oracle.OracleGraph.from_graph(g)
    w = og.weights(delta)
    assert w.W == p * q + q * r
    assert og.brute_count(M40, delta) == p * q * r
    assert og.exhaustive(w, M40)[1] == p * q * r


def test_gadget_estimator_binomial():
    """G1 (r = 1): X is 1 on the p*q closing paths and 0 on the q others, so
    hits ~ Bin(k, p/(p+1)) and C_hat = W * hits / k."""
    p, q = 4, 3
    g, delta = sg.gen_gadget(p, q, 1)
    og = oracle.OracleGraph.from_graph(g)
    w = og.weights(delta)
    k = 200000
    e = og.sample(w, [M40], k, seed=5)
    hits = int(e.hits[0])
    assert e.cnt[0] == hits
    pr = p / (p + 1)
    z = (hits - k * pr) / math.sqrt(k * pr * (1 - pr))
    assert abs(z) < 5
    assert e.est[0] == (hits / k) * w.W


# ------------------------------------------------------------ sampler ------
def test_sampler_uniform_over_paths():
    """Lemma "sample": each delta-centred path has probability 1/W."""
    g = sg.gen_micro(4, n=5, m=20, t_span=8)
    delta = 4
    og = oracle.OracleGraph.from_graph(g)
    w = og.weights(delta)
    paths = brute.enumerate_paths(g.src, g.dst, g.t, delta)
    assert w.W == len(paths) and 20 <= w.W <= 400
    index = {p: i for i, p in enumerate(paths)}
    k = 400000
    e = og.sample(w, [M40], k, seed=9, per_sample=True)
    ids = np.array([index[(int(a), int(b), int(c))] for a, b, c in zip(e.e1, e.e2, e.e3)])
    obs = np.bincount(ids, minlength=len(paths))
    exp = k / len(paths)
    chi2 = ((obs - exp) ** 2 / exp).sum()
    dof = len(paths) - 1
    assert chi2 < dof + 6 * math.sqrt(2 * dof)


def test_estimator_unbiased_over_seeds():
    """Claim "est": E[C_hat] = C; z-test with the exact Var[X] from
    exhaustive enumeration of all paths."""
    g = sg.gen_tiny()
    delta = 20000
    og = oracle.OracleGraph.from_graph(g)
    w = og.weights(delta)
    st, sx, sx2, _ = og.exhaustive(w, M40)
    C = og.brute_count(M40, delta)
    assert sx == C and C > 100
    W = w.W
    var_x = sx2 / W - (sx / W) ** 2
    k, seeds = 20000, 40
    ests = [og.sample(w, [M40], k, seed=s).est[0] for s in range(1, seeds + 1)]
    se = W * math.sqrt(var_x / (k * seeds))
    z = (np.mean(ests) - C) / se
    assert abs(z) < 4.5, (np.mean(ests), C, se)


def test_chunked_sampling_equals_one_shot():
    g = sg.gen_tiny()
    og = oracle.OracleGraph.from_graph(g)
    w = og.weights(20000)
    motifs = [sg.motif_bytes(sg.MOTIFS[n]) for n in sg.SIX_MOTIFS]
    full = og.sample(w, motifs, 30000, seed=3, stream=2, per_sample=True)
    parts = [og.sample(w, motifs, 10000, seed=3, stream=2, i0=i0, per_sample=True)
             for i0 in (0, 10000, 20000)]
    for j in range(len(motifs)):
        assert full.cnt[j] == sum(p.cnt[j] for p in parts)
        assert np.array_equal(full.X[j], np.concatenate([p.X[j] for p in parts]))
    assert np.array_equal(full.e1, np.concatenate([p.e1 for p in parts]))


def test_delta_zero_gives_zero():
    g = sg.gen_tiny()
    og = oracle.OracleGraph.from_graph(g)
    w = og.weights(0)
    e = og.sample(w, [M40], 1000, seed=1)
    assert og.brute_count(M40, 0) == 0
    assert e.cnt[0] == 0 and e.est[0] == 0.0


def test_zero_weight_graph():
    src = np.array([0, 2], np.int32)
    dst = np.array([1, 3], np.int32)
    t = np.array([5, 6], np.int64)
    og = oracle.OracleGraph(4, src, dst, t)
    w = og.weights(100)
    assert w.W == 0
    e = og.sample(w, [M40], 50, seed=1, per_sample=True)
    assert e.status == 0 and e.est[0] == 0.0 and e.cnt[0] == 0
    assert (e.e1 == -1).all() and (e.X == 0).all()


def test_range_errors():
    with pytest.raises(ValueError):
        oracle.OracleGraph(3, np.array([0], np.int32), np.array([3], np.int32), np.array([0], np.int64))
    with pytest.raises(ValueError):
        oracle.OracleGraph(3, np.array([0], np.int32), np.array([1], np.int32), np.array([2**62], np.int64))
    og = oracle.OracleGraph(3, np.array([0], np.int32), np.array([1], np.int32),
                            np.array([2**62 - 1], np.int64))
    assert og.weights(2**62).status == 0


def test_weight_total_overflow_detected():
    """Three layers of 2^21, 2^22, 2^21 parallel edges: W = 2^64 exactly, one
    fewer middle edge gives 2^64 - 2^42 with no overflow."""
    g = sg.gen_overflow_layers(2**21, 2**22, 2**21)
    og = oracle.OracleGraph.from_graph(g)
    w = og.weights(0)
    assert w.status == oracle.OR_OVERFLOW
    del og
    g = sg.gen_overflow_layers(2**21, 2**22 - 1, 2**21)
    og = oracle.OracleGraph.from_graph(g)
    w = og.weights(0)
    assert w.status == 0 and w.W == 2**64 - 2**42
