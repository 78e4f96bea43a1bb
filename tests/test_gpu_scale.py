"""Parity at the Bitcoin-like scale (5*10^7 vertices, 3*10^8 edges, hubs with
more than 10^6 edges): the paths that only this size reaches -- 26-bit vertex
ids (four passes per vertex sort), a 28-bit time range, an eight-level search
tree over S with its top levels cached in LDS, a 2^29-slot pair-run table and
pair runs of hub vertices -- against the oracle, on the graph and launch
shape the benchmark times.  Every order, offset, window and S is compared
entry by entry; every per-sample output of a 2*10^5-sample window per delta
(the six motifs), and of a window whose counters straddle i = 2^32."""
import os

import numpy as np
import pytest

import synthgraph as sg
from test_gpu_parity import _u32, _u64

pytestmark = pytest.mark.gpu

SIX = [sg.MOTIFS[n] for n in sg.SIX_MOTIFS]


@pytest.fixture(scope="module")
def big():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import oracle
    import paper_2409_08975_amd as tcb
    g = sg.gen_bitcoin_like()
    s, d, t = (torch.from_numpy(g.src).cuda(), torch.from_numpy(g.dst).cuda(),
               torch.from_numpy(g.t).cuda())
    G = tcb.tc_build_graph(g.n, s, d, t, check=True)
    threads = min(len(os.sched_getaffinity(0)), int(os.environ.get("OMP_NUM_THREADS", "16")))
    og = oracle.OracleGraph.from_graph(g, threads=max(1, threads))
    yield tcb, g, G, og, max(1, threads)
    del G, og
    torch.cuda.empty_cache()


def test_bitcoin_scale_orders_and_offsets(big):
    tcb, g, G, og, th = big
    A = G.arrays()
    o = og.orders()
    for name in ("out_eid", "in_eid", "pair_eid"):
        assert np.array_equal(A[name].cpu().numpy(), o[name]), name
    assert np.array_equal(_u32(A["out_off"]), o["out_off"])
    assert np.array_equal(_u32(A["in_off"]), o["in_off"])
    oe = o["out_eid"]
    assert np.array_equal(A["out_t"].cpu().numpy(), g.t[oe])
    assert np.array_equal(A["out_dst"].cpu().numpy(), g.dst[oe])
    pe = o["pair_eid"]
    assert np.array_equal(A["pair_t"].cpu().numpy(), g.t[pe])
    # the hubs are there: some vertex has more than 10^6 out-edges
    assert int(np.diff(o["out_off"].astype(np.int64)).max()) > 10**6
    assert G.c.pair_hash_log2 == 29


@pytest.mark.parametrize("delta", [3600, 86400])
def test_bitcoin_scale_weights_and_samples(big, delta):
    tcb, g, G, og, th = big
    W = tcb.tc_path_weights(G, delta)
    ow = og.weights(delta, threads=th)
    A = W.arrays()
    assert W.status() == 0 == ow.status
    for name in ("lo_in", "a", "lo_out", "b"):
        assert np.array_equal(_u32(A[name]), getattr(ow, name)), name
    assert np.array_equal(_u64(A["S"]), ow.S)
    mb = [sg.motif_bytes(M) for M in SIX]
    for k, seed, stream, i0 in ((200000, 1, 0, 0), (50000, 7, 5, (1 << 32) - 20000)):
        R = tcb.tc_sample_estimate(G, W, SIX, k, seed, stream, i0, per_sample=True)
        E = og.sample(ow, mb, k, seed, stream, i0, per_sample=True, threads=th)
        st = int(R.status.item()) & 0xFFFFFFFF
        assert st == E.status
        assert np.array_equal(R.e1.cpu().numpy(), E.e1)
        assert np.array_equal(R.e2.cpu().numpy(), E.e2)
        assert np.array_equal(R.e3.cpu().numpy(), E.e3)
        assert np.array_equal(R.P.cpu().numpy().view(np.uint32), E.P)
        assert np.array_equal(_u64(R.X), E.X)
        if st == 0:
            assert R.counts() == E.cnt
            assert np.array_equal(R.estimate.cpu().numpy().view(np.uint64), E.est.view(np.uint64))
    del W, ow
