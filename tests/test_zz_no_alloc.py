"""The no-allocation sampler entry point (tc_sample_estimate_noalloc, scratch
in the library's static per-GPU array) against tc_sample_estimate (caller
workspace) on the same inputs: two calls in a row, the second smaller, so
that the second must not be confused by what the first left in the shared
scratch.  Integer results and per-sample outputs bit for bit, the estimate
bit-identical."""
import numpy as np
import pytest

import synthgraph as sg

pytestmark = pytest.mark.gpu

SIX = [sg.MOTIFS[n] for n in sg.SIX_MOTIFS]


@pytest.fixture(scope="module")
def tcb():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2409_08975_amd as tcb
    tcb.lib()
    return tcb


def _u64(t):
    return t.cpu().numpy().view(np.uint64)


def _same(a, b):
    assert int(a.status.item()) == int(b.status.item())
    assert a.counts() == b.counts()
    assert np.array_equal(_u64(a.hits), _u64(b.hits))
    assert np.array_equal(a.estimate.cpu().numpy().view(np.uint64),
                          b.estimate.cpu().numpy().view(np.uint64))
    for f in ("e1", "e2", "e3"):
        assert np.array_equal(getattr(a, f).cpu().numpy(), getattr(b, f).cpu().numpy()), f
    assert np.array_equal(_u64(a.X), _u64(b.X))


def _graph(tcb, g):
    import torch
    return tcb.tc_build_graph(g.n, torch.from_numpy(g.src).cuda(), torch.from_numpy(g.dst).cuda(),
                              torch.from_numpy(g.t).cuda(), check=True)


def test_noalloc_equals_workspace_call_twice(tcb):
    import torch
    # first call: the tiny workload, six motifs, 200,000 samples (four chunks
    # of the no-allocation launch shape)
    g1 = sg.gen_tiny()
    G1 = _graph(tcb, g1)
    W1 = tcb.tc_path_weights(G1, 20000)
    k1, seed1 = 200000, 9
    a = tcb.tc_sample_estimate_noalloc(G1, W1, SIX, k1, seed1, 2, 17, per_sample=True)
    b = tcb.tc_sample_estimate(G1, W1, SIX, k1, seed1, 2, 17, per_sample=True)
    torch.cuda.synchronize()
    a.check()
    _same(a, b)
    assert sum(a.counts()) > 0
    # the oracle agrees too
    import oracle
    og = oracle.OracleGraph.from_graph(g1)
    E = og.sample(og.weights(20000), [sg.motif_bytes(M) for M in SIX], k1, seed1, 2, 17)
    assert E.status == 0 and a.counts() == E.cnt
    # second call, smaller: a planted micro graph, one motif, 3,000 samples
    g2 = sg.gen_micro_planted(3, sg.MOTIFS["M4-0"], copies=4, n=7, noise=10)
    G2 = _graph(tcb, g2)
    W2 = tcb.tc_path_weights(G2, 9)
    k2, seed2 = 3000, 4
    a2 = tcb.tc_sample_estimate_noalloc(G2, W2, [sg.MOTIFS["M4-0"]], k2, seed2, per_sample=True)
    b2 = tcb.tc_sample_estimate(G2, W2, [sg.MOTIFS["M4-0"]], k2, seed2, per_sample=True)
    torch.cuda.synchronize()
    a2.check()
    _same(a2, b2)
    assert a2.counts()[0] > 0


def test_noalloc_argument_errors(tcb):
    import torch
    g = sg.gen_micro(3, n=6, m=40, t_span=10)
    G = _graph(tcb, g)
    W = tcb.tc_path_weights(G, 5)
    with pytest.raises(tcb.TCError) as e:
        tcb.tc_sample_estimate_noalloc(G, W, [[(0, 1), (1, 2), (2, 3)]] * 17, 10, 1)
    assert e.value.code == tcb.TC_E_ARG
    with pytest.raises(tcb.TCError) as e:
        # a 3-star: no 3-path to anchor on
        tcb.tc_sample_estimate_noalloc(G, W, [[(0, 1), (0, 2), (0, 3)]], 10, 1)
    assert e.value.code == tcb.TC_E_UNSUPPORTED
    torch.cuda.synchronize()
