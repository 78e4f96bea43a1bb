"""Seeded synthetic temporal multigraphs and the motif catalogue.

This module is the single source of inputs for both the CPU oracle and the
HIP path.  It holds none of the estimator's arithmetic: it only draws edge
lists (src, dst, t) and spells out motif edge lists.

Input model (the paper's datasets are not available, so these stand in for
their shapes; see the experiments section, dataset table):

* Vertex popularity follows a Chung-Lu power law: the vertex of popularity
  rank r gets weight (r+1)^(-1/(alpha-1)), which yields a degree
  distribution with exponent alpha.  One random permutation assigns ranks to
  vertex ids and is shared by the source and destination roles, so in-hubs
  are also out-hubs and directed cycles exist.
* src and dst are drawn independently from those weights; a self-loop is
  redrawn on the destination side.
* Timestamps are int64 seconds.

Directed temporal multigraph conventions follow the problem definition
(section I-A): edges are (u, v, t), parallel edges are allowed, the edge id
(eid) of an edge is its index in the input arrays.
"""
from __future__ import annotations

import dataclasses
import numpy as np

__all__ = [
    "TemporalGraph", "MOTIFS", "SIX_MOTIFS", "motif_bytes", "gen_tiny",
    "gen_medium", "gen_micro", "gen_bitcoin_like", "zipf_vertex_weights",
    "TINY", "MEDIUM",
]


@dataclasses.dataclass
class TemporalGraph:
    n: int
    src: np.ndarray  # int32 [m]
    dst: np.ndarray  # int32 [m]
    t: np.ndarray    # int64 [m]
    name: str = ""

    @property
    def m(self) -> int:
        return int(self.src.shape[0])


# ---------------------------------------------------------------------------
# Motif catalogue.  Each motif is its edge list in pi order (edge i has time
# rank i) over vertices A=0, B=1, C=2, D=3.  Ranks 0,1,2 are the directed
# 3-path A->B->C->D that serves as the anchor.
#   M4-0: the simple temporal 4-cycle (section II figure list; text in the
#         introduction and insights paragraphs).
#   M4-1: the 9-edge pattern spelled out in the CheckMotif discussion
#         (section III-B): (A,B,0),(B,C,1),(C,D,2),(D,C,3),(C,B,4),(B,A,5),
#         (A,B,6),(B,C,7),(C,D,8).
#   The remaining four are stand-ins: the figures that define M4-2..M4-5 are
#   not available, so these are chosen to exercise the same machinery
#   (repeated pairs, chords, a second lap, a 10-edge pattern with every pair
#   doubled).
# ---------------------------------------------------------------------------
A, B, C, D = 0, 1, 2, 3
_SPINE = [(A, B), (B, C), (C, D)]
MOTIFS = {
    "M4-0": _SPINE + [(D, A)],
    "M4-1": _SPINE + [(D, C), (C, B), (B, A), (A, B), (B, C), (C, D)],
    "S3-cycle2": _SPINE + [(D, A), (A, B), (B, C), (C, D), (D, A)],
    "S4-chord": _SPINE + [(D, A), (A, C)],
    "S5-paw": _SPINE + [(D, B)],
    "S6-double": _SPINE + [(D, A), (A, C), (A, B), (B, C), (C, D), (D, A), (A, C)],
}
SIX_MOTIFS = list(MOTIFS.keys())


def motif_bytes(edges, nv: int = 4) -> bytes:
    """Pack a motif as the 34-byte descriptor {u8 nv, u8 ne, u8 src[16], u8 dst[16]}."""
    ne = len(edges)
    if ne > 16:
        raise ValueError("at most 16 motif edges")
    s = bytearray(34)
    s[0] = nv
    s[1] = ne
    for i, (a, b) in enumerate(edges):
        s[2 + i] = a
        s[18 + i] = b
    return bytes(s)


def zipf_vertex_weights(n: int, alpha: float, rng: np.random.Generator) -> np.ndarray:
    """Chung-Lu weights for degree exponent alpha, permuted onto vertex ids."""
    ranks = np.arange(1, n + 1, dtype=np.float64)
    w = ranks ** (-1.0 / (alpha - 1.0))
    perm = rng.permutation(n)
    out = np.empty(n, dtype=np.float64)
    out[perm] = w
    return out / out.sum()


def _draw_endpoints(n, m, p, rng):
    cdf = np.cumsum(p)
    cdf[-1] = 1.0
    src = np.searchsorted(cdf, rng.random(m), side="right").astype(np.int32)
    dst = np.searchsorted(cdf, rng.random(m), side="right").astype(np.int32)
    np.minimum(src, n - 1, out=src)
    np.minimum(dst, n - 1, out=dst)
    loops = np.nonzero(src == dst)[0]
    while loops.size:
        dst[loops] = np.minimum(
            np.searchsorted(cdf, rng.random(loops.size), side="right"), n - 1)
        loops = loops[src[loops] == dst[loops]]
    return src, dst


# Tiny workload: 2,000 vertices, 20,000 edges, Zipf(2.1) weights, no
# self-loops, ~10% of edges repeat the (u, v) pair of an earlier edge,
# timestamps uniform in [0, 10^6]; delta = 3,600; M4-0; k = 10^5.
TINY = dict(n=2000, m=20000, alpha=2.1, repeat_frac=0.10, t_max=10**6,
            delta=3600, k=10**5, seed=1)


def gen_tiny(seed: int = 1001, n: int = TINY["n"], m: int = TINY["m"],
             alpha: float = TINY["alpha"], repeat_frac: float = TINY["repeat_frac"],
             t_max: int = TINY["t_max"]) -> TemporalGraph:
    rng = np.random.default_rng(seed)
    p = zipf_vertex_weights(n, alpha, rng)
    src, dst = _draw_endpoints(n, m, p, rng)
    # ~repeat_frac of the edges copy the pair of a uniformly chosen earlier
    # fresh edge (a multigraph with repeated pairs).
    rep = rng.random(m) < repeat_frac
    rep[0] = False
    fresh_idx = np.nonzero(~rep)[0]
    for i in np.nonzero(rep)[0]:
        cand = fresh_idx[fresh_idx < i]
        j = cand[rng.integers(0, cand.size)]
        src[i] = src[j]
        dst[i] = dst[j]
    t = rng.integers(0, t_max + 1, size=m, dtype=np.int64)
    return TemporalGraph(n, src, dst, t, name="tiny")


# Medium workload: 10^6 vertices, 2*10^7 edges, Zipf(2.1), bursty timestamps
# over a 30-day span: 10^6 burst centres uniform over the span, each edge
# joins a uniform burst (mean 20 edges per burst) at an offset floor(Exp(tau))
# seconds, tau = 600 s, clipped to the span; delta = 86,400; six motifs;
# k = 10^7.
MEDIUM = dict(n=10**6, m=2 * 10**7, alpha=2.1, span=30 * 86400, bursts=10**6,
              tau=600.0, delta=86400, k=10**7, seed=1)


def gen_medium(seed: int = 1002, n: int = MEDIUM["n"], m: int = MEDIUM["m"],
               alpha: float = MEDIUM["alpha"], span: int = MEDIUM["span"],
               bursts: int = MEDIUM["bursts"], tau: float = MEDIUM["tau"]) -> TemporalGraph:
    rng = np.random.default_rng(seed)
    p = zipf_vertex_weights(n, alpha, rng)
    src, dst = _draw_endpoints(n, m, p, rng)
    centres = rng.integers(0, span, size=bursts, dtype=np.int64)
    which = rng.integers(0, bursts, size=m)
    off = np.floor(rng.exponential(tau, size=m)).astype(np.int64)
    t = np.minimum(centres[which] + off, span - 1)
    return TemporalGraph(n, src, dst, t, name="medium")


def _powerlaw_ranks(rng, size: int, n: int, beta: float) -> np.ndarray:
    """Ranks in [0, n) with density proportional to (r + 1)^-beta: inverse of
    the continuous CDF F(x) = ((x + 1)^(1 - beta) - 1) / ((n + 1)^(1 - beta) - 1)."""
    a = 1.0 - beta
    top = (n + 1.0) ** a - 1.0
    r = np.floor((1.0 + rng.random(size) * top) ** (1.0 / a) - 1.0).astype(np.int64)
    return np.minimum(r, n - 1)


def gen_bitcoin_like(seed: int = 1003, n: int = 5 * 10**7, m: int = 3 * 10**8,
                     alpha: float = 1.9, span: int = 7 * 365 * 86400,
                     chunk: int = 1 << 24) -> TemporalGraph:
    """Bitcoin-like scale: endpoint ranks drawn from a power law with degree
    exponent alpha (rank density (r + 1)^(-1 / (alpha - 1)), one random
    permutation mapping ranks to vertex ids for both roles, no self-loops),
    each drawn (u, v) pair repeated Geometric(0.5) times, timestamps uniform
    over seven years at 1 s."""
    rng = np.random.default_rng(seed)
    beta = 1.0 / (alpha - 1.0)
    perm = rng.permutation(n).astype(np.int32)
    src = np.empty(m, dtype=np.int32)
    dst = np.empty(m, dtype=np.int32)
    filled = 0
    while filled < m:
        q = min(chunk, m - filled)
        s = _powerlaw_ranks(rng, q, n, beta)
        d = _powerlaw_ranks(rng, q, n, beta)
        loops = np.nonzero(s == d)[0]
        while loops.size:
            d[loops] = _powerlaw_ranks(rng, loops.size, n, beta)
            loops = loops[s[loops] == d[loops]]
        reps = rng.geometric(0.5, size=q)
        s = np.repeat(perm[s], reps)
        d = np.repeat(perm[d], reps)
        take = min(s.size, m - filled)
        src[filled:filled + take] = s[:take]
        dst[filled:filled + take] = d[:take]
        filled += take
    t = rng.integers(0, span, size=m, dtype=np.int64)
    return TemporalGraph(n, src, dst, t, name="bitcoin-like")


BITCOIN = dict(n=5 * 10**7, m=3 * 10**8, alpha=1.9, span=7 * 365 * 86400,
               deltas=[600, 3600, 86400, 604800], k=10**8, seed=1)


def gen_micro(seed: int, n: int = 5, m: int = 16, t_span: int = 12,
              allow_self_loops: bool = False) -> TemporalGraph:
    """Very small dense graphs with many ties and repeated pairs, for
    exhaustive checks against the definition of a match."""
    rng = np.random.default_rng(seed)
    src = rng.integers(0, n, size=m).astype(np.int32)
    dst = rng.integers(0, n, size=m).astype(np.int32)
    if not allow_self_loops:
        loops = src == dst
        dst[loops] = (dst[loops] + 1 + rng.integers(0, n - 1, size=int(loops.sum()))) % n
    t = rng.integers(0, t_span + 1, size=m).astype(np.int64)
    return TemporalGraph(n, src.astype(np.int32), dst.astype(np.int32), t, name=f"micro{seed}")


def gen_micro_planted(seed: int, motif_edges, copies: int = 3, n: int = 6,
                      noise: int = 8, t_span: int = 20) -> TemporalGraph:
    """Micro graph with `copies` time-increasing instances of a motif planted
    on random vertex 4-tuples (with jittered, sometimes tied, times) plus
    `noise` random edges; used for exhaustive checks where matches exist."""
    rng = np.random.default_rng(seed)
    src, dst, t = [], [], []
    for _ in range(copies):
        phi = rng.permutation(n)[:4]
        base = int(rng.integers(0, max(1, t_span // 2)))
        tt = base
        for (a, b) in motif_edges:
            tt += int(rng.choice([0, 1, 2], p=[0.1, 0.45, 0.45]))  # 0 makes a tie: not a match
            src.append(int(phi[a]))
            dst.append(int(phi[b]))
            t.append(tt)
    for _ in range(noise):
        s = int(rng.integers(0, n))
        d = int((s + 1 + rng.integers(0, n - 1)) % n)
        src.append(s)
        dst.append(d)
        t.append(int(rng.integers(0, t_span + 1)))
    order = rng.permutation(len(src))
    return TemporalGraph(n, np.asarray(src, np.int32)[order], np.asarray(dst, np.int32)[order],
                         np.asarray(t, np.int64)[order], name=f"planted{seed}")


def gen_gadget(p: int, q: int, r: int = 1):
    """Closed-form gadget: p edges A->B at times 1..p, one B->C at p+1, q
    edges C->D at p+2..p+q+1, r edges D->A at p+q+2..p+q+r+1, with
    delta = p+q+r+1.  The 4-cycle count is p*q*r and the number of
    delta-centred <-,+,<,>> 3-paths is p*q + q*r."""
    A_, B_, C_, D_ = 0, 1, 2, 3
    src = [A_] * p + [B_] + [C_] * q + [D_] * r
    dst = [B_] * p + [C_] + [D_] * q + [A_] * r
    t = list(range(1, p + 1)) + [p + 1] + list(range(p + 2, p + q + 2)) + \
        list(range(p + q + 2, p + q + r + 2))
    delta = p + q + r + 1
    return TemporalGraph(4, np.asarray(src, np.int32), np.asarray(dst, np.int32),
                         np.asarray(t, np.int64), name=f"gadget{p}x{q}x{r}"), delta


def gen_overflow_layers(l1: int, l2: int, l3: int) -> TemporalGraph:
    """Three layers of parallel edges x->u, u->v, v->y, all at time 0: every
    u->v edge sees l1 in-edges and l3 out-edges, so the total path weight is
    l1 * l2 * l3 (used to drive the weight total to and past 2^64)."""
    src = np.concatenate([np.full(l1, 0), np.full(l2, 1), np.full(l3, 2)]).astype(np.int32)
    dst = np.concatenate([np.full(l1, 1), np.full(l2, 2), np.full(l3, 3)]).astype(np.int32)
    t = np.zeros(l1 + l2 + l3, np.int64)
    return TemporalGraph(4, src, dst, t, name="overflow-layers")


def relabel_spread(g: TemporalGraph, n_new: int, seed: int) -> TemporalGraph:
    """The same edges with vertex ids mapped injectively onto random ids in
    [0, n_new) (n_new >= g.n): exercises wide vertex ids (more radix passes,
    large offset arrays) on a small edge list."""
    rng = np.random.default_rng(seed)
    ids = np.sort(rng.choice(n_new, size=g.n, replace=False)).astype(np.int32)
    rng.shuffle(ids)
    return TemporalGraph(n_new, ids[g.src], ids[g.dst], g.t.copy(), name=g.name + "-spread")


def random_bf16_bits(seed: int, shape, exp_lo: int = 118, exp_hi: int = 129) -> np.ndarray:
    """bfloat16 bit patterns (uint16) with random sign, a biased exponent in
    [exp_lo, exp_hi] and random 7-bit mantissa: magnitudes roughly
    2^(exp_lo-127) .. 2^(exp_hi-126).  Inputs for network tests."""
    rng = np.random.default_rng(seed)
    n = int(np.prod(shape))
    sign = rng.integers(0, 2, size=n, dtype=np.uint16) << 15
    expo = rng.integers(exp_lo, exp_hi + 1, size=n).astype(np.uint16) << 7
    mant = rng.integers(0, 128, size=n, dtype=np.uint16)
    return (sign | expo | mant).astype(np.uint16).reshape(shape)


def random_params(seed: int, n: int = 4801, scale: float = 0.25) -> np.ndarray:
    """float32 normal parameters for network tests."""
    rng = np.random.default_rng(seed)
    return (rng.standard_normal(n) * scale).astype(np.float32)


def random_counts(seed: int, n: int, p_nonzero: float = 0.3) -> np.ndarray:
    """uint64 per-sample counts: zero with probability 1 - p_nonzero, else
    1 + Geometric-like small integers."""
    rng = np.random.default_rng(seed)
    x = rng.geometric(0.5, size=n).astype(np.uint64)
    x[rng.random(n) >= p_nonzero] = 0
    return x
