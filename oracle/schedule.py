"""Plain reference of the two scheduling rules around the tile operation --
test infrastructure only (see the package docstring for who may import it).

1. Dependency trees (Sec. 3.1.1).  A tile's tree is a multiset of arrivals
   (generation g, children c), the background tile being the one arrival of
   generation 0.  Generation 0 expects one tile; generation g + 1 expects the
   sum of the children declared by the tiles of generation g.  Writing n(g)
   for the arrivals of generation g and E(g) for what it expects, the state
   of a multiset is, scanning g = 0, 1, 2, ... past the largest generation:
     - "error"    at the first g with n(g) > E(g), all earlier generations
                  holding exactly what they expect;
     - "waiting"  at the first g with n(g) < E(g), likewise;
     - "complete" if every generation holds exactly what it expects (the scan
                  then ends at a generation that expects nothing).
   Arrivals may come in any generation order (Sec. 3.1.1), so the state of an
   arrival sequence is the state of the multiset of its prefix.

2. Variance-driven assignment of extra samples (Sec. 4.1.1: tiles with a
   higher variance are rendered by more ranks).  Reading: ``extra`` renders
   are apportioned to the tiles in proportion to the tile variance by the
   largest-remainder (Hamilton) method: quotas q_t = extra w_t / S with
   w_t = v_t where finite and positive, else 0, and S the sum of w_t in tile
   order; each tile gets floor(q_t), the renders left over go one each to the
   largest remainders q_t - floor(q_t), ties to the smaller tile id; S = 0
   gives the uniform split, the remainder to the first tiles.  The floating
   point steps are fixed (double, sum in tile order, (extra * w_t) / S) so
   that every implementation takes the same integer decisions.
"""
from __future__ import annotations

import math
from collections import Counter, defaultdict

WAITING, COMPLETE, ERROR = "waiting", "complete", "error"


def tree_progress(arrivals):
    """(state, generation, missing) of one tile's tree given the multiset of
    (generation, children) arrivals, the background tile included as
    generation 0: the scan stops at the generation that decides the state;
    missing is what a waiting generation still lacks (else 0); a complete
    tree reports its last generation."""
    n = Counter(int(g) for g, _ in arrivals)
    declared = defaultdict(int)
    for g, c in arrivals:
        declared[int(g)] += int(c)
    top = max(n) + 1 if n else 1
    last = None
    for g in range(top + 1):
        expect = 1 if g == 0 else declared[g - 1]
        if n[g] > expect:
            return ERROR, g, 0
        if n[g] < expect:
            return WAITING, g, expect - n[g]
        if expect == 0 and last is None:  # the generation after the last one
            last = g - 1
    return COMPLETE, last, 0


def tree_state(arrivals):
    return tree_progress(arrivals)[0]


def tree_trace(arrivals):
    """State after each prefix of an arrival sequence."""
    return [tree_state(arrivals[:i + 1]) for i in range(len(arrivals))]


def assign_samples(variance, extra):
    """Largest-remainder apportionment of ``extra`` renders (rule 2 above).
    ``variance``: per-tile float32 values; returns a list of ints."""
    T = len(variance)
    w = []
    for v in variance:
        v = float(v)
        w.append(v if math.isfinite(v) and v > 0.0 else 0.0)
    S = 0.0
    for x in w:
        S += x
    if not S > 0.0:
        base, rest = divmod(extra, T)
        return [base + (1 if t < rest else 0) for t in range(T)]
    q = [extra * x / S for x in w]
    c = [math.floor(v) for v in q]
    left = extra - sum(c)
    by_remainder = sorted(range(T), key=lambda t: (-(q[t] - c[t]), t))
    for t in by_remainder[:left]:
        c[t] += 1
    return c
