"""Python binding of libtc.so (the MI355X temporal 3-path sampling library).

Argument marshalling only: every step of the path runs in the HIP kernels of
``libtc.so``.  PyTorch provides device memory and the current HIP stream.
The names mirror the C ABI in ``include/tc.h``.  The library must be built
(``python paper_2409_08975_amd/build.py``); importing the binding without it
raises, and there is no CPU fallback.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass, field

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libtc.so")

TC_OK, TC_E_ARG, TC_E_RANGE, TC_E_OVERFLOW, TC_E_UNSUPPORTED, TC_E_WORKSPACE, TC_E_HIP = (
    0, -1, -2, -3, -4, -5, -6)
TC_F_RANGE, TC_F_OVERFLOW, TC_F_RNG = 1, 2, 4


def TC_F_MOTIF(j: int) -> int:
    """Status bit naming motif j of a call whose count reached 2^64."""
    return 1 << (8 + j)
_STATUS_NAMES = {0: "TC_OK", -1: "TC_E_ARG", -2: "TC_E_RANGE", -3: "TC_E_OVERFLOW",
                 -4: "TC_E_UNSUPPORTED", -5: "TC_E_WORKSPACE", -6: "TC_E_HIP"}

EXPORTED = ["tc_version", "tc_graph_workspace_bytes", "tc_build_graph",
            "tc_weights_workspace_bytes", "tc_path_weights", "tc_path_weights_class",
            "tc_weights_batch_workspace_bytes", "tc_path_weights_batch",
            "tc_motif_anchor", "tc_exhaustive_count", "tc_sample_workspace_bytes",
            "tc_sample_estimate", "tc_sample_estimate_noalloc", "tc_batch_workspace_bytes", "tc_batch_estimate",
            "tc_autotune", "tc_features_workspace_bytes", "tc_edge_features", "tc_mlp_forward", "tc_mlp_workspace_bytes",
            "tc_mlp_grad", "tc_mlp_adam", "tc_mlp_train", "tc_quantize_proposal",
            "tc_proposal_workspace_bytes", "tc_proposal_weights", "tc_window_factors",
            "tc_proposal_window_workspace_bytes", "tc_proposal_window", "tc_timing_enable",
            "tc_timing_reset", "tc_timing_read"]
MLP_PARAMS = 4801


class TCError(RuntimeError):
    def __init__(self, code, what=""):
        self.code = code
        super().__init__(f"{what}: {_STATUS_NAMES.get(code, code)}")


class TCDeviceError(RuntimeError):
    def __init__(self, bits, what=""):
        self.bits = bits
        names = [n for b, n in ((TC_F_RANGE, "RANGE"), (TC_F_OVERFLOW, "OVERFLOW"),
                                (TC_F_RNG, "RNG")) if bits & b]
        motifs = [j for j in range(16) if bits & (1 << (8 + j))]
        if motifs:
            names.append("motifs " + ",".join(map(str, motifs)))
        super().__init__(f"{what}: device status {'|'.join(names) or bits}")


_P = ctypes.c_void_p


class tc_motif(ctypes.Structure):
    _fields_ = [("nv", ctypes.c_uint8), ("ne", ctypes.c_uint8),
                ("src", ctypes.c_uint8 * 16), ("dst", ctypes.c_uint8 * 16)]


TC_SIDE_NONE, TC_SIDE_IN, TC_SIDE_OUT = 0, 1, 2
TC_WINDOW_OPEN = 2  # added to an `after` value: the window leaves out the centre time


class tc_class(ctypes.Structure):
    """Anchor class: side 1 (at the centre's source u) and side 3 (at its
    destination v), each with a mode (none / in-edge / out-edge) and whether
    its edge comes after the centre (plus TC_WINDOW_OPEN for a window open at
    the centre time)."""
    _fields_ = [("mode1", ctypes.c_uint8), ("after1", ctypes.c_uint8),
                ("mode3", ctypes.c_uint8), ("after3", ctypes.c_uint8)]

    def as_tuple(self):
        return (self.mode1, self.after1, self.mode3, self.after3)


SPINE_CLASS = (TC_SIDE_IN, 0, TC_SIDE_OUT, 1)


class tc_graph(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32), ("m", ctypes.c_int64), ("t_range", _P),
                ("out_off", _P), ("out_src", _P), ("out_dst", _P),
                ("out_eid", _P), ("out_t", _P), ("in_off", _P), ("in_src", _P), ("in_eid", _P),
                ("in_dst", _P), ("in_t", _P), ("pair_dst", _P),
                ("pair_eid", _P), ("pair_t", _P),
                ("status", _P), ("pair_hash", _P), ("pair_hash_log2", ctypes.c_int32),
                ("out_rec", _P), ("in_rec", _P), ("pair_skip", _P)]


class tc_weights(ctypes.Structure):
    _fields_ = [("delta", ctypes.c_int64), ("m", ctypes.c_int64), ("lo_in", _P), ("a", _P),
                ("lo_out", _P), ("b", _P), ("S", _P), ("status", _P), ("scratch", _P),
                ("h", _P), ("prec", _P), ("cls", tc_class), ("ps1", _P), ("ps3", _P)]


class tc_result(ctypes.Structure):
    _fields_ = [("cnt", _P), ("hits", _P), ("estimate", _P), ("status", _P), ("e1", _P),
                ("e2", _P), ("e3", _P), ("X", _P), ("P", _P), ("m2", _P), ("xmax", _P)]


class tc_tuning(ctypes.Structure):
    _fields_ = [("chunk_log2", ctypes.c_int32), ("path_blocks", ctypes.c_int32),
                ("reg_waves", ctypes.c_int32), ("fast_waves", ctypes.c_int32),
                ("wide_blocks", ctypes.c_int32), ("reg_list_cap", ctypes.c_int32),
                ("lds_list_cap", ctypes.c_int32)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


def make_tuning(chunk_log2=25, path_blocks=0, reg_waves=40960, fast_waves=8192,
                wide_blocks=2048, reg_list_cap=256, lds_list_cap=1024) -> tc_tuning:
    return tc_tuning(chunk_log2, path_blocks, reg_waves, fast_waves, wide_blocks, reg_list_cap,
                     lds_list_cap)


_lib = None


def lib():
    """Load libtc.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with paper_2409_08975_amd/build.py")
        L = ctypes.CDLL(LIB_PATH)
        I32, I64, U64, U32, SZ = (ctypes.c_int32, ctypes.c_int64, ctypes.c_uint64,
                                  ctypes.c_uint32, ctypes.c_size_t)
        L.tc_version.restype = ctypes.c_char_p
        L.tc_graph_workspace_bytes.argtypes = [I32, I64, ctypes.POINTER(SZ)]
        L.tc_build_graph.argtypes = [I32, I64, _P, _P, _P, _P, SZ, _P, ctypes.POINTER(tc_graph)]
        L.tc_weights_workspace_bytes.argtypes = [I64, ctypes.POINTER(SZ)]
        L.tc_path_weights.argtypes = [ctypes.POINTER(tc_graph), I64, _P, SZ, _P,
                                      ctypes.POINTER(tc_weights)]
        L.tc_path_weights_class.argtypes = [ctypes.POINTER(tc_graph), I64,
                                            ctypes.POINTER(tc_class), _P, SZ, _P,
                                            ctypes.POINTER(tc_weights)]
        L.tc_weights_batch_workspace_bytes.argtypes = [I64, I32, ctypes.POINTER(SZ)]
        L.tc_path_weights_batch.argtypes = [ctypes.POINTER(tc_graph), _P, I32,
                                            ctypes.POINTER(tc_class), _P, SZ, _P, _P]
        L.tc_motif_anchor.argtypes = [ctypes.POINTER(tc_motif), ctypes.POINTER(tc_class),
                                      ctypes.POINTER(I32), ctypes.POINTER(I32)]
        L.tc_exhaustive_count.argtypes = [ctypes.POINTER(tc_graph), ctypes.POINTER(tc_weights),
                                          ctypes.POINTER(tc_motif), I32, U64, U64, _P, SZ,
                                          ctypes.POINTER(tc_result), _P]
        L.tc_sample_workspace_bytes.argtypes = [U64, I32, ctypes.POINTER(SZ)]
        L.tc_sample_estimate.argtypes = [ctypes.POINTER(tc_graph), ctypes.POINTER(tc_weights),
                                         ctypes.POINTER(tc_motif), I32, U64, U64, U32, U64,
                                         _P, SZ, ctypes.POINTER(tc_result), _P]
        L.tc_sample_estimate_noalloc.argtypes = [ctypes.POINTER(tc_graph),
                                                 ctypes.POINTER(tc_weights),
                                                 ctypes.POINTER(tc_motif), I32, U64, U64, U32,
                                                 U64, ctypes.POINTER(tc_result), _P]
        L.tc_batch_workspace_bytes.argtypes = [U64, I32, I32, ctypes.POINTER(SZ)]
        L.tc_batch_estimate.argtypes = [ctypes.POINTER(tc_graph), _P, I32,
                                        ctypes.POINTER(tc_motif), I32, U64, U64, U32, U64,
                                        ctypes.POINTER(tc_tuning), _P, SZ, _P, _P]
        L.tc_autotune.argtypes = [ctypes.POINTER(tc_graph), _P, I32, ctypes.POINTER(tc_motif),
                                  I32, U64, U64, _P, SZ, _P, _P, ctypes.POINTER(tc_tuning),
                                  ctypes.POINTER(ctypes.c_double)]
        F32 = ctypes.c_float
        L.tc_features_workspace_bytes.argtypes = [I64, ctypes.POINTER(SZ)]
        L.tc_edge_features.argtypes = [ctypes.POINTER(tc_graph), ctypes.POINTER(tc_weights), _P,
                                       _P, SZ, _P]
        L.tc_mlp_forward.argtypes = [_P, _P, I64, _P, _P]
        L.tc_mlp_workspace_bytes.argtypes = [I64, ctypes.POINTER(SZ)]
        L.tc_mlp_grad.argtypes = [_P, _P, I64, _P, _P, I64, F32, _P, _P, _P, SZ, _P]
        L.tc_mlp_adam.argtypes = [_P, _P, _P, I64, F32, _P]
        L.tc_mlp_train.argtypes = [_P, _P, _P, I64, _P, _P, I64, F32, I32, I32, F32, U64, I64, _P,
                                   _P, SZ, _P]
        L.tc_quantize_proposal.argtypes = [ctypes.POINTER(tc_weights), _P, F32, _P, _P, _P]
        L.tc_proposal_workspace_bytes.argtypes = [I64, ctypes.POINTER(SZ)]
        L.tc_proposal_weights.argtypes = [ctypes.POINTER(tc_graph), ctypes.POINTER(tc_weights),
                                          _P, _P, SZ, ctypes.POINTER(tc_weights), _P]
        L.tc_window_factors.argtypes = [ctypes.POINTER(tc_graph), I32, U32, _P, _P, _P]
        L.tc_proposal_window_workspace_bytes.argtypes = [I64, ctypes.POINTER(SZ)]
        L.tc_proposal_window.argtypes = [ctypes.POINTER(tc_graph), ctypes.POINTER(tc_weights),
                                         _P, _P, _P, _P, SZ, ctypes.POINTER(tc_weights), _P]
        L.tc_timing_enable.argtypes = [I32]
        L.tc_timing_reset.argtypes = []
        L.tc_timing_read.argtypes = [ctypes.c_char_p, ctypes.POINTER(ctypes.c_double),
                                     ctypes.POINTER(I64)]
        for name in EXPORTED[1:]:
            getattr(L, name).restype = ctypes.c_int
        _lib = L
    return _lib


def _check(code, what):
    if code != TC_OK:
        raise TCError(code, what)


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else ctypes.c_void_p(0)


def _stream(stream=None):
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _on_stream(stream, *tensors):
    """Tie tensors allocated on the current stream to the explicit stream
    their kernels are enqueued on, so the caching allocator does not hand
    their memory to other work before those kernels are done."""
    if stream is not None:
        for t in tensors:
            if t is not None:
                t.record_stream(stream)


def make_motif(edges, nv: int | None = None) -> tc_motif:
    """Motif descriptor of an edge list in pi order; nv defaults to the
    number of vertices the edges use (3 or 4)."""
    m = tc_motif()
    m.nv = nv if nv is not None else 1 + max(max(a, b) for a, b in edges)
    m.ne = len(edges)
    for i, (a, b) in enumerate(edges):
        m.src[i] = a
        m.dst[i] = b
    return m


@dataclass
class Graph:
    c: tc_graph
    ws: torch.Tensor
    inputs: tuple = field(default=())

    @property
    def n(self):
        return self.c.n

    @property
    def m(self):
        return self.c.m

    def status(self):
        """The build's device status word (TC_F_* bits; synchronises)."""
        return int(self.view("status", torch.int32, 1).item()) & 0xFFFFFFFF

    def check(self, what="tc_build_graph"):
        """Raise TCDeviceError if the build rejected its input (synchronises)."""
        s = self.status()
        if s:
            raise TCDeviceError(s, what)
        return self

    def time_range(self):
        """(t_min, t_max) of the input, from the device (synchronises)."""
        tr = self.view("t_range", torch.int64, 2).cpu().tolist()
        return tr[0], tr[1]

    def view(self, name, dtype, length):
        """Tensor view of one device array of the graph (no copy)."""
        ptr = getattr(self.c, name)
        base = self.ws.data_ptr()
        elt = torch.empty((), dtype=dtype).element_size()
        off = ptr - base
        return self.ws[off:off + length * elt].view(dtype)

    def arrays(self):
        n, m = self.n, self.m
        d = {}
        for name, dt, ln in [("out_off", torch.int32, n + 1), ("in_off", torch.int32, n + 1),
                             ("out_src", torch.int32, m), ("out_dst", torch.int32, m),
                             ("out_eid", torch.int32, m), ("out_t", torch.int64, m),
                             ("in_src", torch.int32, m), ("in_eid", torch.int32, m),
                             ("in_dst", torch.int32, m), ("in_t", torch.int64, m),
                             ("pair_dst", torch.int32, m),
                             ("pair_eid", torch.int32, m), ("pair_t", torch.int64, m)]:
            d[name] = self.view(name, dt, ln)
        return d


@dataclass
class Weights:
    c: tc_weights
    ws: torch.Tensor
    graph: Graph
    base: "Weights | None" = None     # the method's weights a proposal set borrows from
    h: torch.Tensor | None = None     # proposal factors (int32 storage of uint32)
    factors: tuple | None = None      # window proposal: (f_in, f_out) it was built from

    def view(self, name, dtype, length):
        ptr = getattr(self.c, name)
        off = ptr - self.ws.data_ptr()
        elt = torch.empty((), dtype=dtype).element_size()
        return self.ws[off:off + length * elt].view(dtype)

    def arrays(self):
        m = self.c.m
        if self.base is not None:
            d = self.base.arrays()
            d["S"] = self.view("S", torch.int64, m + 1)
            return d
        return dict(lo_in=self.view("lo_in", torch.int32, m), a=self.view("a", torch.int32, m),
                    lo_out=self.view("lo_out", torch.int32, m), b=self.view("b", torch.int32, m),
                    S=self.view("S", torch.int64, m + 1))

    def status(self) -> int:
        return int(self.view("status", torch.int32, 1).item()) & 0xFFFFFFFF

    def total(self) -> int:
        """W_delta as a Python int (synchronises)."""
        return int(self.view("S", torch.int64, self.c.m + 1)[-1].item()) & (2**64 - 1)


@dataclass
class Result:
    cnt: torch.Tensor       # int64 [2 * n_motifs] (lo, hi) bit patterns of u64
    hits: torch.Tensor      # int64 [n_motifs]
    estimate: torch.Tensor  # float64 [n_motifs]
    status: torch.Tensor    # int32 [1]
    e1: torch.Tensor | None = None
    e2: torch.Tensor | None = None
    e3: torch.Tensor | None = None
    X: torch.Tensor | None = None  # int64 [n_motifs, k] (u64 bit patterns)
    P: torch.Tensor | None = None  # int32 [k] centre scan positions (u32 bit patterns)
    m2: torch.Tensor | None = None  # float64 [n_motifs] sum of (X / h)^2
    xmax: torch.Tensor | None = None  # int64 [n_motifs] largest X (u64 bit patterns)

    def counts(self):
        c = self.cnt.cpu().tolist()
        return [(c[2 * j] & (2**64 - 1)) | ((c[2 * j + 1] & (2**64 - 1)) << 64)
                for j in range(len(c) // 2)]

    def check(self, what="tc_sample_estimate"):
        s = int(self.status.item()) & 0xFFFFFFFF
        if s:
            raise TCDeviceError(s, what)
        return self


def graph_workspace_bytes(n: int, m: int) -> int:
    b = ctypes.c_size_t(0)
    _check(lib().tc_graph_workspace_bytes(n, m, ctypes.byref(b)), "tc_graph_workspace_bytes")
    return b.value


def weights_workspace_bytes(m: int) -> int:
    b = ctypes.c_size_t(0)
    _check(lib().tc_weights_workspace_bytes(m, ctypes.byref(b)), "tc_weights_workspace_bytes")
    return b.value


def weights_batch_workspace_bytes(m: int, n_deltas: int) -> int:
    b = ctypes.c_size_t(0)
    _check(lib().tc_weights_batch_workspace_bytes(m, int(n_deltas), ctypes.byref(b)),
           "tc_weights_batch_workspace_bytes")
    return b.value


def sample_workspace_bytes(k: int, n_motifs: int) -> int:
    b = ctypes.c_size_t(0)
    _check(lib().tc_sample_workspace_bytes(int(k), int(n_motifs), ctypes.byref(b)),
           "tc_sample_workspace_bytes")
    return b.value


def batch_workspace_bytes(k: int, n_deltas: int, n_motifs: int) -> int:
    b = ctypes.c_size_t(0)
    _check(lib().tc_batch_workspace_bytes(int(k), int(n_deltas), int(n_motifs), ctypes.byref(b)),
           "tc_batch_workspace_bytes")
    return b.value


_ws_cache: dict = {}


def _sample_ws(k: int, nm: int, device, nd: int = 1, stream=None) -> torch.Tensor:
    """Scratch for the sampler, kept per (device, stream) and grown on demand
    (stream-ordered reuse)."""
    need = batch_workspace_bytes(k, nd, nm)
    st = stream if stream is not None else torch.cuda.current_stream(device)
    key = (str(device), st.cuda_stream)
    buf = _ws_cache.get(key)
    if buf is None or buf.numel() < need:
        buf = torch.empty(need, dtype=torch.uint8, device=device)
        _ws_cache[key] = buf
    return buf


def tc_build_graph(n: int, src: torch.Tensor, dst: torch.Tensor, t: torch.Tensor,
                   stream=None, check: bool = False,
                   workspace: torch.Tensor | None = None) -> Graph:
    """Build the temporal adjacency on the device (inputs: int32, int32, int64
    CUDA tensors).  Enqueue only; with check=True the call waits for the
    validation and raises TCDeviceError on a bad vertex id or time."""
    assert src.is_cuda and dst.is_cuda and t.is_cuda
    assert src.dtype == torch.int32 and dst.dtype == torch.int32 and t.dtype == torch.int64
    src, dst, t = src.contiguous(), dst.contiguous(), t.contiguous()
    m = src.numel()
    assert dst.numel() == m and t.numel() == m
    nbytes = graph_workspace_bytes(n, m)
    if workspace is not None:
        assert workspace.numel() >= nbytes
        ws = workspace
    else:
        ws = torch.empty(nbytes, dtype=torch.uint8, device=src.device)
    g = tc_graph()
    _on_stream(stream, ws, src, dst, t)
    _check(lib().tc_build_graph(n, m, _ptr(src), _ptr(dst), _ptr(t), _ptr(ws), nbytes,
                                _stream(stream), ctypes.byref(g)), "tc_build_graph")
    G = Graph(g, ws, (src, dst, t))
    return G.check() if check else G


def tc_path_weights(graph: Graph, delta: int, stream=None,
                    workspace: torch.Tensor | None = None, cls=None) -> Weights:
    """Preprocess(delta) for an anchor class (a tuple (mode1, after1, mode3,
    after3) or a tc_class; default: the <-,+,<,>> class)."""
    nbytes = weights_workspace_bytes(graph.m)
    if workspace is not None:
        assert workspace.numel() >= nbytes
        ws = workspace
    else:
        ws = torch.empty(nbytes, dtype=torch.uint8, device=graph.ws.device)
    w = tc_weights()
    _on_stream(stream, ws)
    if cls is None:
        _check(lib().tc_path_weights(ctypes.byref(graph.c), int(delta), _ptr(ws), nbytes,
                                     _stream(stream), ctypes.byref(w)), "tc_path_weights")
    else:
        c = cls if isinstance(cls, tc_class) else tc_class(*cls)
        _check(lib().tc_path_weights_class(ctypes.byref(graph.c), int(delta), ctypes.byref(c),
                                           _ptr(ws), nbytes, _stream(stream), ctypes.byref(w)),
               "tc_path_weights_class")
    return Weights(w, ws, graph)


def tc_path_weights_batch(graph: Graph, deltas, stream=None,
                          workspace: torch.Tensor | None = None, cls=None) -> list:
    """Preprocess for several deltas of one anchor class in one launch
    sequence; returns one Weights per delta (all in one workspace)."""
    nd = len(deltas)
    nbytes = weights_batch_workspace_bytes(graph.m, nd)
    if workspace is not None:
        assert workspace.numel() >= nbytes
        ws = workspace
    else:
        ws = torch.empty(nbytes, dtype=torch.uint8, device=graph.ws.device)
    ds = (ctypes.c_int64 * nd)(*[int(d) for d in deltas])
    ws_arr = (tc_weights * nd)()
    c = None
    if cls is not None:
        c = cls if isinstance(cls, tc_class) else tc_class(*cls)
    _on_stream(stream, ws)
    _check(lib().tc_path_weights_batch(ctypes.byref(graph.c), ds, nd,
                                       ctypes.byref(c) if c is not None else None, _ptr(ws),
                                       nbytes, _stream(stream), ws_arr), "tc_path_weights_batch")
    out = []
    for i in range(nd):
        out.append(Weights(tc_weights.from_buffer_copy(ws_arr[i]), ws, graph))
    return out


def tc_motif_anchor(edges, nv: int | None = None):
    """(class tuple, number of anchor edges, their rank order) of a motif's
    anchor; raises TCError(TC_E_UNSUPPORTED) if it has none."""
    m = make_motif(edges, nv)
    c = tc_class()
    na = ctypes.c_int32(0)
    order = (ctypes.c_int32 * 3)()
    _check(lib().tc_motif_anchor(ctypes.byref(m), ctypes.byref(c), ctypes.byref(na), order),
           "tc_motif_anchor")
    return c.as_tuple(), na.value, list(order)[:na.value]


def new_result(n_motifs: int, k: int, device, per_sample: bool = False,
               moments: bool = False) -> Result:
    """Output buffers of one delta (per-sample arrays only with per_sample,
    the second moment only with moments)."""
    nm = n_motifs
    out = Result(torch.zeros(2 * nm, dtype=torch.int64, device=device),
                 torch.zeros(nm, dtype=torch.int64, device=device),
                 torch.zeros(nm, dtype=torch.float64, device=device),
                 torch.zeros(1, dtype=torch.int32, device=device))
    if per_sample:
        out.e1 = torch.empty(k, dtype=torch.int32, device=device)
        out.e2 = torch.empty(k, dtype=torch.int32, device=device)
        out.e3 = torch.empty(k, dtype=torch.int32, device=device)
        out.X = torch.empty((nm, k), dtype=torch.int64, device=device)
        out.P = torch.empty(k, dtype=torch.int32, device=device)
    if moments:
        out.m2 = torch.zeros(nm, dtype=torch.float64, device=device)
    out.xmax = torch.zeros(nm, dtype=torch.int64, device=device)
    return out


def _c_result(out: Result) -> tc_result:
    return tc_result(_ptr(out.cnt).value, _ptr(out.hits).value, _ptr(out.estimate).value,
                     _ptr(out.status).value, _ptr(out.e1).value, _ptr(out.e2).value,
                     _ptr(out.e3).value, _ptr(out.X).value, _ptr(out.P).value,
                     _ptr(out.m2).value, _ptr(out.xmax).value)


def _motif_array(motifs):
    """Motifs as edge lists (vertex count inferred) or (edges, nv) pairs."""
    nm = len(motifs)
    ms = [make_motif(m[0], m[1]) if isinstance(m, tuple) and len(m) == 2 and
          isinstance(m[1], int) else make_motif(m) for m in motifs]
    return nm, (tc_motif * nm)(*ms)


def tc_sample_estimate(graph: Graph, weights: Weights, motifs, k: int, seed: int,
                       stream_id: int = 0, i0: int = 0, per_sample: bool = False,
                       stream=None, out: Result | None = None,
                       workspace: torch.Tensor | None = None, moments: bool = False) -> Result:
    """Estimate(M, k) for a list of motifs (each a list of (src, dst) edges in
    pi order); importance sampling when `weights` is a proposal set."""
    nm, arr = _motif_array(motifs)
    dev = graph.ws.device
    if out is None:
        out = new_result(nm, k, dev, per_sample, moments)
        _on_stream(stream, out.cnt, out.hits, out.estimate, out.status, out.e1, out.e2, out.e3,
                   out.X, out.P, out.m2)
    r = _c_result(out)
    ws = _sample_ws(k, nm, dev, 1, stream) if workspace is None else workspace
    _check(lib().tc_sample_estimate(ctypes.byref(graph.c), ctypes.byref(weights.c), arr, nm,
                                    int(k), int(seed), int(stream_id), int(i0), _ptr(ws),
                                    ws.numel(), ctypes.byref(r), _stream(stream)),
           "tc_sample_estimate")
    return out


def tc_exhaustive_count(graph: Graph, weights: Weights, motifs, r0: int = 0,
                        count: int | None = None, per_sample: bool = False, stream=None,
                        out: Result | None = None,
                        workspace: torch.Tensor | None = None) -> Result:
    """Exhaustive mode: CheckMotif over the anchors of CDF ranks r0 .. r0 +
    count - 1 (all W of them by default: W is read from the device); cnt is
    then the exact count, hits / m2 / xmax give the B statistics."""
    nm, arr = _motif_array(motifs)
    if count is None:
        count = max(1, weights.total() - r0)
    dev = graph.ws.device
    if out is None:
        out = new_result(nm, count, dev, per_sample, moments=True)
        _on_stream(stream, out.cnt, out.hits, out.estimate, out.status, out.e1, out.e2, out.e3,
                   out.X, out.P, out.m2, out.xmax)
    r = _c_result(out)
    ws = _sample_ws(count, nm, dev, 1, stream) if workspace is None else workspace
    _check(lib().tc_exhaustive_count(ctypes.byref(graph.c), ctypes.byref(weights.c), arr, nm,
                                     int(r0), int(count), _ptr(ws), ws.numel(), ctypes.byref(r),
                                     _stream(stream)), "tc_exhaustive_count")
    return out


def tc_sample_estimate_noalloc(graph: Graph, weights: Weights, motifs, k: int, seed: int,
                               stream_id: int = 0, i0: int = 0, per_sample: bool = False,
                               stream=None, out: Result | None = None) -> Result:
    """tc_sample_estimate on the library's static per-GPU scratch (no
    workspace is allocated for the call)."""
    nm, arr = _motif_array(motifs)
    if out is None:
        out = new_result(nm, k, graph.ws.device, per_sample)
        _on_stream(stream, out.cnt, out.hits, out.estimate, out.status, out.e1, out.e2, out.e3,
                   out.X, out.P)
    r = _c_result(out)
    _check(lib().tc_sample_estimate_noalloc(ctypes.byref(graph.c), ctypes.byref(weights.c), arr,
                                            nm, int(k), int(seed), int(stream_id), int(i0),
                                            ctypes.byref(r), _stream(stream)),
           "tc_sample_estimate_noalloc")
    return out


class _BatchArgs:
    """ctypes arrays of one batched call, kept alive together."""

    def __init__(self, weights, outs):
        nd = len(weights)
        self.wc = [w.c for w in weights]
        self.wp = (ctypes.POINTER(tc_weights) * nd)(*[ctypes.pointer(c) for c in self.wc])
        self.rc = [_c_result(o) for o in outs]
        self.rp = (ctypes.POINTER(tc_result) * nd)(*[ctypes.pointer(c) for c in self.rc])


def tc_batch_estimate(graph: Graph, weights, motifs, k: int, seed: int, stream_id: int = 0,
                      i0: int = 0, per_sample: bool = False, tuning: tc_tuning | None = None,
                      stream=None, outs=None, workspace: torch.Tensor | None = None):
    """Estimate(M, k) for every motif and every delta of `weights` (a list of
    Weights of this graph) in one launch sequence; returns one Result per delta."""
    nd = len(weights)
    nm, arr = _motif_array(motifs)
    dev = graph.ws.device
    if outs is None:
        outs = [new_result(nm, k, dev, per_sample) for _ in range(nd)]
        for o in outs:
            _on_stream(stream, o.cnt, o.hits, o.estimate, o.status, o.e1, o.e2, o.e3, o.X, o.P)
    args = _BatchArgs(weights, outs)
    ws = _sample_ws(k, nm, dev, nd, stream) if workspace is None else workspace
    _check(lib().tc_batch_estimate(ctypes.byref(graph.c), ctypes.cast(args.wp, _P), nd, arr, nm,
                                   int(k), int(seed), int(stream_id), int(i0),
                                   ctypes.byref(tuning) if tuning is not None else None,
                                   _ptr(ws), ws.numel(), ctypes.cast(args.rp, _P),
                                   _stream(stream)),
           "tc_batch_estimate")
    return outs


def tc_autotune(graph: Graph, weights, motifs, k_probe: int, seed: int = 1, stream=None):
    """Fastest tuning for this (graph, deltas, motifs) by timed probes of
    k_probe samples; returns (tc_tuning, milliseconds of the best probe)."""
    nd = len(weights)
    nm, arr = _motif_array(motifs)
    dev = graph.ws.device
    outs = [new_result(nm, k_probe, dev) for _ in range(nd)]
    args = _BatchArgs(weights, outs)
    ws = _sample_ws(k_probe, nm, dev, nd, stream)
    best = tc_tuning()
    ms = ctypes.c_double(0.0)
    _check(lib().tc_autotune(ctypes.byref(graph.c), ctypes.cast(args.wp, _P), nd, arr, nm,
                             int(k_probe), int(seed), _ptr(ws), ws.numel(),
                             ctypes.cast(args.rp, _P), _stream(stream), ctypes.byref(best),
                             ctypes.byref(ms)),
           "tc_autotune")
    return best, ms.value


# ------------------------------------------------------- learned proposal ----
def tc_edge_features(graph: Graph, weights: Weights, stream=None) -> torch.Tensor:
    """[m, 8] bfloat16 features (int16 storage of the bit patterns)."""
    feat = torch.empty((graph.m, 8), dtype=torch.int16, device=graph.ws.device)
    b = ctypes.c_size_t(0)
    _check(lib().tc_features_workspace_bytes(graph.m, ctypes.byref(b)),
           "tc_features_workspace_bytes")
    ws = torch.empty(b.value, dtype=torch.uint8, device=graph.ws.device)
    _on_stream(stream, feat, ws)
    _check(lib().tc_edge_features(ctypes.byref(graph.c), ctypes.byref(weights.c), _ptr(feat),
                                  _ptr(ws), b.value, _stream(stream)), "tc_edge_features")
    return feat


def tc_mlp_forward(params: torch.Tensor, feat: torch.Tensor, n: int | None = None,
                   stream=None, out: torch.Tensor | None = None) -> torch.Tensor:
    n = feat.shape[0] if n is None else n
    g = torch.empty(n, dtype=torch.float32, device=feat.device) if out is None else out
    _on_stream(stream, g)
    _check(lib().tc_mlp_forward(_ptr(params), _ptr(feat), int(n), _ptr(g), _stream(stream)),
           "tc_mlp_forward")
    return g


def mlp_workspace_bytes(n: int) -> int:
    b = ctypes.c_size_t(0)
    _check(lib().tc_mlp_workspace_bytes(int(n), ctypes.byref(b)), "tc_mlp_workspace_bytes")
    return b.value


def tc_mlp_grad(params, feat, rows, X, n: int | None = None, label_cap: float = 0.0,
                stream=None):
    """(grad [4801] float32, loss [1] float32) of the mean BCE over n labels."""
    n = X.shape[0] if n is None else n
    dev = feat.device
    grad = torch.empty(MLP_PARAMS, dtype=torch.float32, device=dev)
    loss = torch.empty(1, dtype=torch.float32, device=dev)
    nb = mlp_workspace_bytes(n)
    ws = torch.empty(nb, dtype=torch.uint8, device=dev)
    _on_stream(stream, grad, loss, ws)
    _check(lib().tc_mlp_grad(_ptr(params), _ptr(feat), int(feat.shape[0]), _ptr(rows), _ptr(X),
                             int(n), float(label_cap), _ptr(grad), _ptr(loss), _ptr(ws), nb,
                             _stream(stream)), "tc_mlp_grad")
    return grad, loss


def tc_mlp_adam(params, opt, grad, step: int, lr: float, stream=None) -> None:
    _check(lib().tc_mlp_adam(_ptr(params), _ptr(opt), _ptr(grad), int(step), float(lr),
                             _stream(stream)), "tc_mlp_adam")


def tc_mlp_train(params, opt, feat, rows, X, batch: int, epochs: int, lr: float, seed: int,
                 step0: int = 0, label_cap: float = 0.0, stream=None) -> torch.Tensor:
    """Train in place; returns the mean loss of each epoch (device float32)."""
    n = X.shape[0]
    dev = feat.device
    losses = torch.empty(epochs, dtype=torch.float32, device=dev)
    nb = mlp_workspace_bytes(batch)
    ws = torch.empty(nb, dtype=torch.uint8, device=dev)
    _on_stream(stream, losses, ws)
    _check(lib().tc_mlp_train(_ptr(params), _ptr(opt), _ptr(feat), int(feat.shape[0]), _ptr(rows),
                              _ptr(X), int(n), float(label_cap), int(batch), int(epochs),
                              float(lr), int(seed), int(step0), _ptr(losses), _ptr(ws),
                              ws.numel(), _stream(stream)), "tc_mlp_train")
    return losses


def tc_quantize_proposal(weights: Weights, g: torch.Tensor, eps: float = 0.1,
                         normalize: bool = False, stream=None) -> torch.Tensor:
    """Integer proposal factors (int32 storage of uint32); with normalize the
    scores are divided by their maximum first."""
    h = torch.empty(weights.c.m, dtype=torch.int32, device=g.device)
    gmax = torch.empty(1, dtype=torch.float32, device=g.device) if normalize else None
    _on_stream(stream, h, gmax)
    _check(lib().tc_quantize_proposal(ctypes.byref(weights.c), _ptr(g), float(eps), _ptr(gmax),
                                      _ptr(h), _stream(stream)), "tc_quantize_proposal")
    return h


def proposal_workspace_bytes(m: int) -> int:
    b = ctypes.c_size_t(0)
    _check(lib().tc_proposal_workspace_bytes(int(m), ctypes.byref(b)),
           "tc_proposal_workspace_bytes")
    return b.value


def tc_proposal_weights(graph: Graph, weights: Weights, h: torch.Tensor,
                        stream=None) -> Weights:
    """Proposal weight set: windows of `weights`, S = scan of a * b * h."""
    h = h.contiguous()
    nb = proposal_workspace_bytes(graph.m)
    ws = torch.empty(nb, dtype=torch.uint8, device=graph.ws.device)
    wq = tc_weights()
    _on_stream(stream, ws, h)
    _check(lib().tc_proposal_weights(ctypes.byref(graph.c), ctypes.byref(weights.c), _ptr(h),
                                     _ptr(ws), nb, ctypes.byref(wq), _stream(stream)),
           "tc_proposal_weights")
    return Weights(wq, ws, graph, base=weights, h=h)


def tc_window_factors(graph: Graph, quarter: int, cap: int, stream=None):
    """Window-proposal factors (f_in over in-CSR positions, f_out over
    out-CSR positions; int32 tensors holding uint32 values): min(cap, about
    (1 + degree of the far endpoint)^(quarter / 4))."""
    dev = graph.ws.device
    f_in = torch.empty(graph.m, dtype=torch.int32, device=dev)
    f_out = torch.empty(graph.m, dtype=torch.int32, device=dev)
    _on_stream(stream, f_in, f_out)
    _check(lib().tc_window_factors(ctypes.byref(graph.c), int(quarter), int(cap), _ptr(f_in),
                                   _ptr(f_out), _stream(stream)), "tc_window_factors")
    return f_in, f_out


def tc_proposal_window(graph: Graph, weights: Weights, h: torch.Tensor | None = None,
                       f_in: torch.Tensor | None = None, f_out: torch.Tensor | None = None,
                       stream=None) -> Weights:
    """Window proposal set: windows of `weights`, S = scan of h * G1 * G3,
    side edges drawn by their entry factors."""
    h = h.contiguous() if h is not None else None
    f_in = f_in.contiguous() if f_in is not None else None
    f_out = f_out.contiguous() if f_out is not None else None
    b = ctypes.c_size_t(0)
    _check(lib().tc_proposal_window_workspace_bytes(graph.m, ctypes.byref(b)),
           "tc_proposal_window_workspace_bytes")
    ws = torch.empty(b.value, dtype=torch.uint8, device=graph.ws.device)
    wq = tc_weights()
    _on_stream(stream, ws, *[x for x in (h, f_in, f_out) if x is not None])
    null = None
    _check(lib().tc_proposal_window(ctypes.byref(graph.c), ctypes.byref(weights.c),
                                    _ptr(h) if h is not None else null,
                                    _ptr(f_in) if f_in is not None else null,
                                    _ptr(f_out) if f_out is not None else null, _ptr(ws), b.value,
                                    ctypes.byref(wq), _stream(stream)), "tc_proposal_window")
    return Weights(wq, ws, graph, base=weights, h=h, factors=(f_in, f_out))


def timing_enable(on: bool = True) -> None:
    _check(lib().tc_timing_enable(1 if on else 0), "tc_timing_enable")


def timing_reset() -> None:
    _check(lib().tc_timing_reset(), "tc_timing_reset")


def timing_read(kernel: str):
    """(total milliseconds, launches) recorded for one kernel."""
    ms = ctypes.c_double(0.0)
    n = ctypes.c_int64(0)
    _check(lib().tc_timing_read(kernel.encode(), ctypes.byref(ms), ctypes.byref(n)),
           "tc_timing_read")
    return ms.value, n.value


def version() -> str:
    return lib().tc_version().decode()
