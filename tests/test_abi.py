"""Host-side checks of the C ABI: the library loads, exports every symbol the
header declares, and host-checkable errors are reported without touching a
GPU (no compute call is made here)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "tc.h")


def _declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(tc_[a-z_0-9]+)\s*\(", src)))


@pytest.fixture(scope="module")
def tcb():
    import paper_2409_08975_amd as tcb
    if not os.path.exists(tcb.LIB_PATH):
        import paper_2409_08975_amd.build as b
        b.build()
    tcb.lib()
    return tcb


def test_header_declares_the_three_phases():
    d = _declared()
    for name in ["tc_build_graph", "tc_path_weights", "tc_sample_estimate",
                 "tc_graph_workspace_bytes", "tc_weights_workspace_bytes", "tc_version"]:
        assert name in d


def test_library_exports_every_declared_symbol(tcb):
    L = tcb.lib()
    for name in _declared():
        assert hasattr(L, name), name
    assert set(_declared()) == set(tcb.EXPORTED)


def test_version_string(tcb):
    assert "gfx950" in tcb.version()


def test_workspace_queries(tcb):
    b1 = tcb.graph_workspace_bytes(1000, 20000)
    b2 = tcb.graph_workspace_bytes(1000, 40000)
    assert b2 > b1 > 20000 * 16
    w = tcb.weights_workspace_bytes(20000)
    assert w >= 20000 * 16 + 20001 * 8
    assert tcb.weights_workspace_bytes(0) > 0
    with pytest.raises(tcb.TCError):
        tcb.graph_workspace_bytes(0, 10)
    with pytest.raises(tcb.TCError):
        tcb.graph_workspace_bytes(10, -1)
    with pytest.raises(tcb.TCError):
        tcb.graph_workspace_bytes(10, 2**31)


def test_sample_workspace_query(tcb):
    b1 = tcb.sample_workspace_bytes(1000, 1)
    b6 = tcb.sample_workspace_bytes(1000, 6)
    big = tcb.sample_workspace_bytes(10**9, 6)
    assert b6 > b1 > 0
    assert big == tcb.sample_workspace_bytes(2**25, 6)  # chunked: bounded in k
    with pytest.raises(tcb.TCError):
        tcb.sample_workspace_bytes(0, 1)
    with pytest.raises(tcb.TCError):
        tcb.sample_workspace_bytes(10, 17)


def test_host_argument_errors_return_before_any_launch(tcb):
    L = tcb.lib()
    g = tcb.tc_graph()
    # n < 1, null workspace
    assert L.tc_build_graph(0, 1, None, None, None, None, 0, None, ctypes.byref(g)) == tcb.TC_E_ARG
    assert L.tc_build_graph(5, 1, None, None, None, ctypes.c_void_p(1), 0, None,
                            ctypes.byref(g)) == tcb.TC_E_ARG
    w = tcb.tc_weights()
    g.m = 10
    w.m = 10
    assert L.tc_path_weights(ctypes.byref(g), -1, ctypes.c_void_p(1), 0, None,
                             ctypes.byref(w)) == tcb.TC_E_ARG
    assert L.tc_path_weights(ctypes.byref(g), 2**62 + 1, ctypes.c_void_p(1), 0, None,
                             ctypes.byref(w)) == tcb.TC_E_ARG
    fake = ctypes.c_void_p(256).value
    r = tcb.tc_result(fake, fake, fake, fake, None, None, None, None)
    bad = [(0, 1), (0, 2), (0, 3)]  # a 3-star: no anchor path
    arr = (tcb.tc_motif * 1)(tcb.make_motif(bad))
    assert L.tc_sample_estimate(ctypes.byref(g), ctypes.byref(w), arr, 1, 10, 1, 0, 0,
                                ctypes.c_void_p(fake), 1 << 40, ctypes.byref(r), None) == tcb.TC_E_UNSUPPORTED
    ok = [(0, 1), (1, 2), (2, 3), (3, 0)]
    arr = (tcb.tc_motif * 1)(tcb.make_motif(ok))
    assert L.tc_sample_estimate(ctypes.byref(g), ctypes.byref(w), arr, 1, 0, 1, 0, 0,
                                ctypes.c_void_p(fake), 1 << 40, ctypes.byref(r), None) == tcb.TC_E_ARG  # k = 0
    assert L.tc_sample_estimate(ctypes.byref(g), ctypes.byref(w), arr, 0, 10, 1, 0, 0,
                                ctypes.c_void_p(fake), 1 << 40, ctypes.byref(r), None) == tcb.TC_E_ARG  # no motifs
    selfloop = [(0, 1), (1, 2), (2, 3), (3, 3)]
    arr = (tcb.tc_motif * 1)(tcb.make_motif(selfloop))
    assert L.tc_sample_estimate(ctypes.byref(g), ctypes.byref(w), arr, 1, 10, 1, 0, 0,
                                ctypes.c_void_p(fake), 1 << 40, ctypes.byref(r), None) == tcb.TC_E_UNSUPPORTED
    r.e1 = fake  # only some per-sample outputs given
    arr = (tcb.tc_motif * 1)(tcb.make_motif(ok))
    assert L.tc_sample_estimate(ctypes.byref(g), ctypes.byref(w), arr, 1, 10, 1, 0, 0,
                                ctypes.c_void_p(fake), 1 << 40, ctypes.byref(r), None) == tcb.TC_E_ARG


def test_anchor_and_class_host_checks(tcb):
    L = tcb.lib()
    assert tcb.tc_motif_anchor([(0, 1), (1, 2), (2, 3), (3, 0)]) == (tcb.SPINE_CLASS, 3, [0, 1, 2])
    # a wedge (3 vertices): base 0 -> 1 first, then 0 -> 2 from 0's out-list
    assert tcb.tc_motif_anchor([(0, 1), (0, 2), (2, 1)]) == ((2, 1, 0, 0), 2, [1, 0])
    with pytest.raises(tcb.TCError) as e:
        tcb.tc_motif_anchor([(0, 1), (0, 2), (0, 3)])
    assert e.value.code == tcb.TC_E_UNSUPPORTED
    g = tcb.tc_graph()
    w = tcb.tc_weights()
    g.m = w.m = 10
    for bad in ((0, 0, 0, 0), (3, 0, 2, 1), (1, 4, 2, 1), (1, 0, 2, 5)):
        c = tcb.tc_class(*bad)
        assert L.tc_path_weights_class(ctypes.byref(g), 5, ctypes.byref(c), ctypes.c_void_p(1), 0,
                                       None, ctypes.byref(w)) == tcb.TC_E_ARG
    # windows open at the centre time are a valid class (the workspace is not)
    for ok in ((1, 2, 2, 1), (1, 0, 2, 3), (2, 3, 0, 0)):
        c = tcb.tc_class(*ok)
        assert L.tc_path_weights_class(ctypes.byref(g), 5, ctypes.byref(c),
                                       ctypes.c_void_p(256), 0, None,
                                       ctypes.byref(w)) == tcb.TC_E_WORKSPACE
    fake = ctypes.c_void_p(256).value
    r = tcb.tc_result(fake, fake, fake, fake, None, None, None, None)
    arr = (tcb.tc_motif * 1)(tcb.make_motif([(0, 1), (1, 2), (2, 3), (3, 0)]))
    assert L.tc_exhaustive_count(ctypes.byref(g), ctypes.byref(w), arr, 1, 0, 0,
                                 ctypes.c_void_p(fake), 1 << 40, ctypes.byref(r),
                                 None) == tcb.TC_E_ARG  # count = 0
    # weights of another class than the motifs' anchors
    w.cls = tcb.tc_class(2, 1, 0, 0)
    assert L.tc_exhaustive_count(ctypes.byref(g), ctypes.byref(w), arr, 1, 0, 5,
                                 ctypes.c_void_p(fake), 1 << 40, ctypes.byref(r),
                                 None) == tcb.TC_E_ARG


def test_binding_raises_without_library(tmp_path, monkeypatch):
    import paper_2409_08975_amd as tcb
    monkeypatch.setattr(tcb, "_lib", None)
    monkeypatch.setattr(tcb, "LIB_PATH", str(tmp_path / "missing.so"))
    with pytest.raises(ImportError):
        tcb.lib()


def test_weights_batch_host_checks(tcb):
    """The batched Preprocess's workspace grows with the number of deltas
    and its argument errors return before anything is enqueued."""
    L = tcb.lib()
    one = tcb.weights_workspace_bytes(20000)
    assert tcb.weights_batch_workspace_bytes(20000, 1) == one
    b2 = tcb.weights_batch_workspace_bytes(20000, 2)
    b8 = tcb.weights_batch_workspace_bytes(20000, 8)
    assert 2 * (one - 20000 * 8) < b2 < 2 * one + 20000 * 16 and b8 > 8 * (one - 20000 * 8)
    for nd in (0, 9):
        with pytest.raises(tcb.TCError):
            tcb.weights_batch_workspace_bytes(100, nd)
    g = tcb.tc_graph()
    g.m = 10
    ws = (tcb.tc_weights * 8)()
    fake = ctypes.c_void_p(256)
    for ds in ([5, -1], [2**62 + 1], [1] * 9):
        arr = (ctypes.c_int64 * len(ds))(*ds)
        assert L.tc_path_weights_batch(ctypes.byref(g), arr, len(ds), None, fake, 1 << 40, None,
                                       ws) == tcb.TC_E_ARG
    arr = (ctypes.c_int64 * 2)(1, 2)
    assert L.tc_path_weights_batch(ctypes.byref(g), arr, 0, None, fake, 1 << 40, None,
                                   ws) == tcb.TC_E_ARG
    c = tcb.tc_class(0, 0, 0, 0)
    assert L.tc_path_weights_batch(ctypes.byref(g), arr, 2, ctypes.byref(c), fake, 1 << 40, None,
                                   ws) == tcb.TC_E_ARG
    assert L.tc_path_weights_batch(None, arr, 2, None, fake, 1 << 40, None, ws) == tcb.TC_E_ARG
    assert L.tc_path_weights_batch(ctypes.byref(g), arr, 2, None, fake, 16, None,
                                   ws) == tcb.TC_E_WORKSPACE


def test_misaligned_workspace_is_an_argument_error(tcb):
    """A workspace must be 256-byte aligned: a misaligned one is refused on
    the host (TC_E_ARG) where an aligned one of the same size gets as far as
    the size check (TC_E_WORKSPACE)."""
    L = tcb.lib()
    g = tcb.tc_graph()
    w = tcb.tc_weights()
    g.m = w.m = 10
    w.cls = tcb.tc_class(*tcb.SPINE_CLASS)
    src = ctypes.c_void_p(4096)
    for base, want in ((256, tcb.TC_E_WORKSPACE), (256 + 16, tcb.TC_E_ARG),
                       (256 + 8, tcb.TC_E_ARG), (4096 + 128, tcb.TC_E_ARG)):
        ws = ctypes.c_void_p(base)
        assert L.tc_build_graph(5, 1, src, src, src, ws, 0, None, ctypes.byref(g)) == want
        g.m = 10
        assert L.tc_path_weights(ctypes.byref(g), 5, ws, 0, None, ctypes.byref(w)) == want
        arr = (ctypes.c_int64 * 2)(1, 2)
        wl = (tcb.tc_weights * 2)()
        assert L.tc_path_weights_batch(ctypes.byref(g), arr, 2, None, ws, 0, None,
                                       wl) == want
        fake = ctypes.c_void_p(256).value
        r = tcb.tc_result(fake, fake, fake, fake, None, None, None, None)
        arr = (tcb.tc_motif * 1)(tcb.make_motif([(0, 1), (1, 2), (2, 3), (3, 0)]))
        assert L.tc_sample_estimate(ctypes.byref(g), ctypes.byref(w), arr, 1, 10, 1, 0, 0, ws,
                                    0, ctypes.byref(r), None) == want
