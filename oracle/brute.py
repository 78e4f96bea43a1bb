"""Pure-Python enumerators written straight from the definitions.

TEST INFRASTRUCTURE ONLY (see the package docstring).  These loops are only
for micro graphs (tens of edges); they pin the C++ oracle.

* ``count_matches``: the definition of an M-match (section I-A).  Because the
  order condition is an "iff" on strict time order, the G-edges of a match
  have pairwise distinct times and, sorted by time, the i-th one is the image
  of the motif edge of rank i.  So every match is a time-increasing
  combination of |E(H)| edges; we enumerate all combinations and test the
  remaining conditions (endpoint map consistent and 1-1, span <= delta).
* ``enumerate_paths``: every delta-centred <-,+,<,>> 3-path (Definitions of a
  delta-centred 3-path and of its class; closed windows as in Claim "count").
* ``enumerate_class_paths``: the same for any anchor class (section III:
  the classes <alpha_1, alpha_3, beta_1, beta_3>; a side may also have no
  edge, which gives the wedges of the 3-vertex case).
* ``list_count_bruteforce``: number of strictly increasing chains across
  lists, by product enumeration.
"""
from __future__ import annotations

import itertools


def count_matches(src, dst, t, motif_edges, delta):
    m = len(src)
    ne = len(motif_edges)
    order = sorted(range(m), key=lambda e: (int(t[e]), e))
    total = 0
    for combo in itertools.combinations(order, ne):
        times = [int(t[e]) for e in combo]
        if any(times[i] >= times[i + 1] for i in range(ne - 1)):
            continue
        if times[-1] - times[0] > delta:
            continue
        phi = {}
        ok = True
        for (ha, hb), e in zip(motif_edges, combo):
            for hv, gv in ((ha, int(src[e])), (hb, int(dst[e]))):
                if phi.setdefault(hv, gv) != gv:
                    ok = False
                    break
            if not ok:
                break
        if not ok:
            continue
        if len(set(phi.values())) != len(phi):
            continue
        total += 1
    return total


def enumerate_paths(src, dst, t, delta):
    """All (e1, e2, e3) with e2 = (u, v, t2), e1 an in-edge of u with
    t1 in [t2 - delta, t2], e3 an out-edge of v with t3 in [t2, t2 + delta]."""
    m = len(src)
    paths = []
    for e2 in range(m):
        u, v, t2 = int(src[e2]), int(dst[e2]), int(t[e2])
        ins = [e for e in range(m) if int(dst[e]) == u and t2 - delta <= int(t[e]) <= t2]
        outs = [e for e in range(m) if int(src[e]) == v and t2 <= int(t[e]) <= t2 + delta]
        for e1 in ins:
            for e3 in outs:
                paths.append((e1, e2, e3))
    return paths


def enumerate_class_paths(src, dst, t, delta, cls):
    """All (e1, e2, e3) of an anchor class given as 4 bytes {mode1, after1,
    mode3, after3}: e2 = (u, v, t2) any edge; e1 an edge at u (mode 1: an
    in-edge x -> u, mode 2: an out-edge u -> x; mode 0: none, e1 = -1) with
    t1 in [t2 - delta, t2] (after1 = 0) or [t2, t2 + delta] (after1 = 1); e3
    likewise at v.  Windows are closed, unless bit 1 of the after byte is set
    (after1 = 2 or 3): then t1 != t2.  e1 and e3 may be any edges (even e2)."""
    m = len(src)

    def side(at, t2, mode, after):
        if mode == 0:
            return [-1]
        lo, hi = (t2, t2 + delta) if after & 1 else (t2 - delta, t2)
        out = []
        for e in range(m):
            ends = int(dst[e]) if mode == 1 else int(src[e])
            te = int(t[e])
            if ends == at and lo <= te <= hi and not (after & 2 and te == t2):
                out.append(e)
        return out

    paths = []
    for e2 in range(m):
        u, v, t2 = int(src[e2]), int(dst[e2]), int(t[e2])
        for e1 in side(u, t2, cls[0], cls[1]):
            for e3 in side(v, t2, cls[2], cls[3]):
                paths.append((e1, e2, e3))
    return paths


def list_count_bruteforce(lists):
    if not lists:
        return 1
    n = 0
    for combo in itertools.product(*lists):
        if all(combo[i] < combo[i + 1] for i in range(len(combo) - 1)):
            n += 1
    return n
