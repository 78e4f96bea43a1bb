"""CPU oracle for the temporal 3-path sampling estimator.

TEST INFRASTRUCTURE ONLY.  Only the tests, ``__graft_entry__.smoke()`` and the
CPU-baseline leg of ``bench.py`` may import this package.  The GPU library
never calls it, and it shares no code with the GPU library: the arithmetic
lives in ``tc_oracle.cpp`` (plain C++17 + OpenMP, built with g++) and in the
pure-Python enumerators of ``brute.py``.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "tc_oracle.cpp")
_LIB = os.path.join(_HERE, "libtc_oracle.so")

OR_OK, OR_RANGE, OR_OVERFLOW, OR_RNG, OR_ARG = 0, 1, 2, 4, 8


def build(force: bool = True) -> str:
    """Compile the oracle with g++ (no HIP)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        cmd = ["g++", "-std=c++17", "-O2", "-fopenmp", "-ffp-contract=off", "-fPIC",
               "-shared", _SRC, "-o", tmp]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        L = ctypes.CDLL(_LIB)
        P, I64, U64, I32, U32 = (ctypes.c_void_p, ctypes.c_int64, ctypes.c_uint64,
                                 ctypes.c_int32, ctypes.c_uint32)
        L.or_graph_new.restype = P
        L.or_graph_new.argtypes = [I32, I64, P, P, P, P, ctypes.c_int]
        L.or_graph_free.argtypes = [P]
        L.or_graph_orders.argtypes = [P, P, P, P, P, P]
        L.or_weights.argtypes = [P, I64, P, P, P, P, P, ctypes.c_int]
        L.or_weights_class.argtypes = [P, I64, P, P, P, P, P, P, ctypes.c_int]
        L.or_anchor.argtypes = [P, P, P, P, P]
        L.or_sample_cls.argtypes = [P, I64, P, P, P, P, P, P, P, P, ctypes.c_int, U64, U64, U32,
                                    U64, P, P, P, P, P, P, P, P, P, P, ctypes.c_int]
        L.or_enumerate.argtypes = [P, I64, P, P, P, P, P, P, P, ctypes.c_int, U64, U64, P, P, P,
                                   P, P, P, P, P, P, ctypes.c_int]
        L.or_check_motif.argtypes = [P, P, I64, I32, I32, I32, P]
        L.or_sample.argtypes = [P, I64, P, P, P, P, P, P, ctypes.c_int, U64, U64, U32, U64,
                                P, P, P, P, P, P, P, ctypes.c_int]
        L.or_sample_ex.argtypes = [P, I64, P, P, P, P, P, P, P, ctypes.c_int, U64, U64, U32,
                                   U64, P, P, P, P, P, P, P, P, P, ctypes.c_int]
        L.or_proposal_scan.argtypes = [P, P, P, P, P]
        L.or_sample_win.argtypes = [P, I64, P, P, P, P, P, P, P, P, P, P, ctypes.c_int, U64, U64,
                                    U32, U64, P, P, P, P, P, P, P, P, P, P, ctypes.c_int]
        L.or_window_factors.argtypes = [P, ctypes.c_int, U32, P, P]
        L.or_proposal_window.argtypes = [P, P, P, P, P, P, P, P, P, P, P, P]
        L.or_features.argtypes = [P, I64, P, P, P, P, P, ctypes.c_int]
        L.or_exhaustive.argtypes = [P, P, I64, P, P, P, P, P, P, P, P, ctypes.c_int]
        L.or_list_lengths.argtypes = [P, P, I64, I32, I32, I32, P]
        L.or_brute_count.argtypes = [P, P, I64, P, ctypes.c_int]
        L.or_list_count.argtypes = [P, P, ctypes.c_int, P]
        L.or_philox4x32_10.argtypes = [P, P, P]
        L.or_lemire64.argtypes = [U64, U64, P]
        L.or_lemire32.argtypes = [U32, U32, P]
        _lib = L
    return _lib


def _p(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


# Anchor classes as 4 bytes {mode1, after1, mode3, after3}: mode 0 = no edge
# on that side, 1 = an in-edge, 2 = an out-edge of the centre's endpoint;
# after 0 = window [t - delta, t], 1 = [t, t + delta].  Side 1 is the centre
# edge's source u, side 3 its destination v.
SIDE_NONE, SIDE_IN, SIDE_OUT = 0, 1, 2
# bit 1 of an `after` byte: the side's window leaves out the centre time
# ([t - delta, t) or (t, t + delta]); every match's anchor still lies in it
WINDOW_OPEN = 2
SPINE_CLASS = bytes([SIDE_IN, 0, SIDE_OUT, 1])  # <-,+,<,>


def class_bytes(mode1, after1, mode3, after3) -> bytes:
    return bytes([mode1, after1, mode3, after3])


def anchor(motif: bytes):
    """(class bytes, number of anchor edges, their rank order as 0 = e1,
    1 = centre, 2 = e3, motif edge of e1 / centre / e3) of a motif's anchor,
    or None if it has none."""
    mb = np.frombuffer(motif, dtype=np.uint8).copy()
    cls = np.zeros(4, np.uint8)
    na = np.zeros(1, np.int32)
    order = np.zeros(3, np.int32)
    ae = np.zeros(3, np.int32)
    if lib().or_anchor(_p(mb), _p(cls), _p(na), _p(order), _p(ae)) != OR_OK:
        return None
    return bytes(cls), int(na[0]), order[:int(na[0])].tolist(), ae.tolist()


def default_threads() -> int:
    return max(1, min(os.cpu_count() or 1, 16))


def philox4x32_10(ctr, key):
    c = np.asarray(ctr, dtype=np.uint32)
    k = np.asarray(key, dtype=np.uint32)
    out = np.zeros(4, dtype=np.uint32)
    lib().or_philox4x32_10(_p(c), _p(k), _p(out))
    return [int(x) for x in out]


def lemire64(x: int, s: int):
    out = np.zeros(1, dtype=np.uint64)
    ok = lib().or_lemire64(x, s, _p(out))
    return (int(out[0]) if ok else None)


def lemire32(x: int, s: int):
    out = np.zeros(1, dtype=np.uint32)
    ok = lib().or_lemire32(x, s, _p(out))
    return (int(out[0]) if ok else None)


def list_count(lists):
    vals = np.concatenate([np.asarray(l, dtype=np.int64) for l in lists]) if lists else np.zeros(0, np.int64)
    off = np.zeros(len(lists) + 1, dtype=np.int64)
    for i, l in enumerate(lists):
        off[i + 1] = off[i] + len(l)
    vals = np.ascontiguousarray(vals)
    X = np.zeros(2, dtype=np.uint64)
    st = lib().or_list_count(_p(vals), _p(off), len(lists), _p(X))
    return st, int(X[0]) | (int(X[1]) << 64)


@dataclass
class Weights:
    delta: int
    lo_in: np.ndarray
    a: np.ndarray
    lo_out: np.ndarray
    b: np.ndarray
    S: np.ndarray
    status: int

    h: np.ndarray | None = None  # proposal h_int per scan position (S is then Q)
    cls: bytes = SPINE_CLASS     # the anchor class of the windows
    ps1: np.ndarray | None = None  # window proposal: prefix sums of side 1's CSR factors
    ps3: np.ndarray | None = None  # ... and of side 3's

    @property
    def W(self) -> int:
        return int(self.S[-1])


@dataclass
class Estimate:
    cnt: list      # python ints (exact)
    hits: np.ndarray
    est: np.ndarray
    status: int
    e1: np.ndarray | None = None
    e2: np.ndarray | None = None
    e3: np.ndarray | None = None
    X: np.ndarray | None = None  # [n_motifs, k]
    P: np.ndarray | None = None  # [k] scan position of the centre edge
    m2: np.ndarray | None = None  # [n_motifs] sum of (X / h)^2
    xmax: np.ndarray | None = None  # [n_motifs] largest X


class OracleGraph:
    """Temporal adjacency of one input graph, built by the oracle."""

    def __init__(self, n: int, src, dst, t, threads: int = 1):
        self.n = int(n)
        self.src = np.ascontiguousarray(src, dtype=np.int32)
        self.dst = np.ascontiguousarray(dst, dtype=np.int32)
        self.t = np.ascontiguousarray(t, dtype=np.int64)
        self.m = int(self.src.shape[0])
        st = ctypes.c_int(0)
        self.h = lib().or_graph_new(self.n, self.m, _p(self.src), _p(self.dst), _p(self.t),
                                    ctypes.byref(st), int(threads))
        self.status = st.value
        if not self.h:
            raise ValueError(f"oracle rejected the graph (status {st.value})")

    @classmethod
    def from_graph(cls, g, threads: int = 1):
        return cls(g.n, g.src, g.dst, g.t, threads)

    def __del__(self):
        h = getattr(self, "h", None)
        if h and _lib is not None:
            _lib.or_graph_free(h)
            self.h = None

    def orders(self):
        m, n = self.m, self.n
        out = np.zeros(m, np.int32)
        inn = np.zeros(m, np.int32)
        pr = np.zeros(m, np.int32)
        oo = np.zeros(n + 1, np.uint32)
        io = np.zeros(n + 1, np.uint32)
        lib().or_graph_orders(self.h, _p(out), _p(inn), _p(pr), _p(oo), _p(io))
        return dict(out_eid=out, in_eid=inn, pair_eid=pr, out_off=oo, in_off=io)

    def weights(self, delta: int, threads: int | None = None, cls: bytes | None = None) -> Weights:
        """Preprocess(delta) for an anchor class (default <-,+,<,>): per scan
        position the two sides' windows (lo1, a) and (lo3, b) and S."""
        m = self.m
        lo_in = np.zeros(m, np.uint32)
        a = np.zeros(m, np.uint32)
        lo_out = np.zeros(m, np.uint32)
        b = np.zeros(m, np.uint32)
        S = np.zeros(m + 1, np.uint64)
        c = np.frombuffer(cls or SPINE_CLASS, dtype=np.uint8).copy()
        st = lib().or_weights_class(self.h, int(delta), _p(c), _p(lo_in), _p(a), _p(lo_out), _p(b),
                                    _p(S), threads or default_threads())
        return Weights(int(delta), lo_in, a, lo_out, b, S, st, None, bytes(cls or SPINE_CLASS))

    def check_motif(self, motif: bytes, delta: int, e1: int, e2: int, e3: int):
        X = np.zeros(1, np.uint64)
        mb = np.frombuffer(motif, dtype=np.uint8).copy()
        st = lib().or_check_motif(self.h, _p(mb), int(delta), e1, e2, e3, _p(X))
        return st, int(X[0])

    def sample(self, w: Weights, motifs, k: int, seed: int, stream: int = 0, i0: int = 0,
               per_sample: bool = False, threads: int | None = None) -> Estimate:
        """Estimate(M, k); with a proposal weight set (w.h set, from
        ``proposal``) the importance-sampling estimator."""
        mb = np.frombuffer(b"".join(motifs), dtype=np.uint8).copy()
        nm = len(motifs)
        cnt = np.zeros(2 * nm, np.uint64)
        hits = np.zeros(nm, np.uint64)
        est = np.zeros(nm, np.float64)
        m2 = np.zeros(nm, np.float64)
        xmax = np.zeros(nm, np.uint64)
        e1 = e2 = e3 = X = P = None
        null = ctypes.c_void_p(0)
        if per_sample:
            e1 = np.zeros(k, np.int32)
            e2 = np.zeros(k, np.int32)
            e3 = np.zeros(k, np.int32)
            X = np.zeros(nm * k, np.uint64)
            P = np.zeros(k, np.uint32)
        hq = _p(w.h) if w.h is not None else null
        c = np.frombuffer(w.cls, dtype=np.uint8).copy()
        p1 = _p(w.ps1) if w.ps1 is not None else null
        p3 = _p(w.ps3) if w.ps3 is not None else null
        st = lib().or_sample_win(self.h, w.delta, _p(c), _p(w.lo_in), _p(w.a), _p(w.lo_out),
                                 _p(w.b), _p(w.S), hq, p1, p3, _p(mb), nm, int(k), int(seed),
                                 int(stream),
                                 int(i0), _p(e1) if per_sample else null,
                                 _p(e2) if per_sample else null, _p(e3) if per_sample else null,
                                 _p(X) if per_sample else null, _p(P) if per_sample else null,
                                 _p(cnt), _p(hits), _p(est), _p(m2), _p(xmax),
                                 threads or default_threads())
        cc = [int(cnt[2 * j]) | (int(cnt[2 * j + 1]) << 64) for j in range(nm)]
        return Estimate(cc, hits, est, st, e1, e2, e3, None if X is None else X.reshape(nm, k),
                        P, m2, xmax)

    def enumerate(self, w: Weights, motifs, r0: int = 0, count: int | None = None,
                  per_sample: bool = False, threads: int | None = None) -> Estimate:
        """Exhaustive mode: CheckMotif over the anchors of ranks r0 .. r0 +
        count - 1 of the integer CDF (all W of them by default); over all of
        them cnt is the exact count C."""
        if count is None:
            count = max(0, w.W - r0)
        mb = np.frombuffer(b"".join(motifs), dtype=np.uint8).copy()
        nm = len(motifs)
        cnt = np.zeros(2 * nm, np.uint64)
        hits = np.zeros(nm, np.uint64)
        est = np.zeros(nm, np.float64)
        m2 = np.zeros(nm, np.float64)
        xmax = np.zeros(nm, np.uint64)
        null = ctypes.c_void_p(0)
        e1 = e2 = e3 = X = None
        if per_sample:
            e1 = np.zeros(count, np.int32)
            e2 = np.zeros(count, np.int32)
            e3 = np.zeros(count, np.int32)
            X = np.zeros(nm * count, np.uint64)
        c = np.frombuffer(w.cls, dtype=np.uint8).copy()
        st = lib().or_enumerate(self.h, w.delta, _p(c), _p(w.lo_in), _p(w.a), _p(w.lo_out),
                                _p(w.b), _p(w.S), _p(mb), nm, int(r0), int(count),
                                _p(e1) if per_sample else null, _p(e2) if per_sample else null,
                                _p(e3) if per_sample else null, _p(X) if per_sample else null,
                                _p(cnt), _p(hits), _p(est), _p(m2), _p(xmax),
                                threads or default_threads())
        cc = [int(cnt[2 * j]) | (int(cnt[2 * j + 1]) << 64) for j in range(nm)]
        return Estimate(cc, hits, est, st, e1, e2, e3,
                        None if X is None else X.reshape(nm, count), None, m2, xmax)

    def proposal(self, w: Weights, h_int) -> Weights:
        """Weight set of the proposal q_p = w_p * h_p: same windows, S = the
        exact scan of q (Q = S[m]), h attached."""
        h = np.ascontiguousarray(h_int, dtype=np.uint32)
        assert h.shape[0] == self.m
        Q = np.zeros(self.m + 1, np.uint64)
        st = lib().or_proposal_scan(self.h, _p(w.a), _p(w.b), _p(h), _p(Q))
        return Weights(w.delta, w.lo_in, w.a, w.lo_out, w.b, Q, st, h, w.cls)

    def window_factors(self, quarter: int, cap: int):
        """Per-entry factors of the window proposal (not part of the paper):
        (f_in over in-CSR positions, f_out over out-CSR positions), each
        min(cap, about (1 + degree of the far endpoint)^(quarter / 4)) in
        integer square roots."""
        f_in = np.zeros(self.m, np.uint32)
        f_out = np.zeros(self.m, np.uint32)
        st = lib().or_window_factors(self.h, int(quarter), int(cap), _p(f_in), _p(f_out))
        if st:
            raise ValueError(f"bad window factor parameters (status {st})")
        return f_in, f_out

    def proposal_window(self, w: Weights, h_int=None, f_in=None, f_out=None) -> Weights:
        """Weight set of the window proposal q_p = h_p * G1_p * G3_p: each
        side's edge is then drawn with probability proportional to its CSR
        entry's factor (f_in for an in-edge side, f_out for an out-edge
        side; None = 1)."""
        null = ctypes.c_void_p(0)
        h = None if h_int is None else np.ascontiguousarray(h_int, dtype=np.uint32)
        fi = None if f_in is None else np.ascontiguousarray(f_in, dtype=np.uint32)
        fo = None if f_out is None else np.ascontiguousarray(f_out, dtype=np.uint32)
        ps_in = np.zeros(self.m + 1, np.uint64) if fi is not None else None
        ps_out = np.zeros(self.m + 1, np.uint64) if fo is not None else None
        Q = np.zeros(self.m + 1, np.uint64)
        c = np.frombuffer(w.cls, dtype=np.uint8).copy()
        st = lib().or_proposal_window(self.h, _p(c), _p(w.lo_in), _p(w.a), _p(w.lo_out), _p(w.b),
                                      _p(h) if h is not None else null,
                                      _p(fi) if fi is not None else null,
                                      _p(fo) if fo is not None else null,
                                      _p(ps_in) if ps_in is not None else null,
                                      _p(ps_out) if ps_out is not None else null, _p(Q))
        mode1, mode3 = w.cls[0], w.cls[2]
        side = {1: ps_in, 2: ps_out, 0: None}
        return Weights(w.delta, w.lo_in, w.a, w.lo_out, w.b, Q, st, h, w.cls,
                       side[mode1], side[mode3])

    def features(self, w: Weights, threads: int | None = None) -> np.ndarray:
        """Per-edge proposal features [m, 8] in binary64 (scan order)."""
        F = np.zeros((self.m, 8), np.float64)
        lib().or_features(self.h, w.delta, _p(w.lo_in), _p(w.a), _p(w.lo_out), _p(w.b), _p(F),
                          threads or default_threads())
        return F

    def exhaustive(self, w: Weights, motif: bytes, threads: int | None = None):
        """Sum over all W delta-centred paths of CheckMotif: (sum X, sum X^2, #X>0)."""
        mb = np.frombuffer(motif, dtype=np.uint8).copy()
        s1 = np.zeros(2, np.uint64)
        s2 = np.zeros(2, np.uint64)
        nz = np.zeros(1, np.uint64)
        c = np.frombuffer(w.cls, dtype=np.uint8).copy()
        st = lib().or_exhaustive(self.h, _p(mb), w.delta, _p(c), _p(w.lo_in), _p(w.a),
                                 _p(w.lo_out), _p(w.b), _p(s1), _p(s2), _p(nz),
                                 threads or default_threads())
        return (st, int(s1[0]) | (int(s1[1]) << 64), int(s2[0]) | (int(s2[1]) << 64), int(nz[0]))

    def list_lengths(self, motif: bytes, delta: int, e1: int, e2: int, e3: int):
        """Window lengths of a path's lists (None if CheckMotif rejects it)."""
        mb = np.frombuffer(motif, dtype=np.uint8).copy()
        lens = np.zeros(16, np.int64)
        n = lib().or_list_lengths(self.h, _p(mb), int(delta), e1, e2, e3, _p(lens))
        return None if n < 0 else lens[:n].tolist()

    def brute_count(self, motif: bytes, delta: int, threads: int | None = None) -> int:
        mb = np.frombuffer(motif, dtype=np.uint8).copy()
        C = np.zeros(2, np.uint64)
        st = lib().or_brute_count(self.h, _p(mb), int(delta), _p(C), threads or default_threads())
        if st:
            raise ValueError(f"brute count failed: {st}")
        return int(C[0]) | (int(C[1]) << 64)
