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


def list_count_bruteforce(lists):
    if not lists:
        return 1
    n = 0
    for combo in itertools.product(*lists):
        if all(combo[i] < combo[i + 1] for i in range(len(combo) - 1)):
            n += 1
    return n
