"""Dependency trees (Sec. 3.1.1) and variance-driven sample assignment
(Sec. 4.1.1): the oracle pinned to constructions and brute force, then the
library's host-side implementations (no GPU involved) checked against it."""
import itertools
import math
import random

import numpy as np
import pytest

from oracle import schedule as orc

COMPLETE, WAITING, ERROR = orc.COMPLETE, orc.WAITING, orc.ERROR


# ------------------------------------------------------------ tree fixtures
def random_tree(rng, max_gen=4, max_children=3):
    """A complete tree built top-down: the background declares c0 children,
    every tile of generation g declares children for g + 1, and exactly the
    declared number of tiles is created for each generation."""
    nodes = []
    c0 = rng.randint(0, max_children)
    nodes.append((0, c0))
    want, g = c0, 1
    while want > 0:
        nxt = 0
        for i in range(want):
            c = rng.randint(0, max_children) if g < max_gen else 0
            nodes.append((g, c))
            nxt += c
        want, g = nxt, g + 1
    return nodes


def figure_tree():
    """The tile pipeline figure: the owner's background tile declares two
    generation-1 tiles, which declare nothing further."""
    return [(0, 2), (1, 0), (1, 0)]


# ------------------------------------------------------------ oracle pins
def test_oracle_tree_figure_example():
    nodes = figure_tree()
    for perm in itertools.permutations(nodes):
        trace = orc.tree_trace(list(perm))
        assert trace[-1] == COMPLETE
        assert all(s == WAITING for s in trace[:-1])
    assert orc.tree_progress([(0, 2), (1, 0)]) == (WAITING, 1, 1)
    assert orc.tree_progress(nodes) == (COMPLETE, 1, 0)


def test_oracle_tree_trivial_cases():
    assert orc.tree_progress([]) == (WAITING, 0, 1)
    assert orc.tree_progress([(0, 0)]) == (COMPLETE, 0, 0)        # background only
    assert orc.tree_state([(0, 0), (0, 0)]) == ERROR               # two backgrounds
    assert orc.tree_state([(0, 0), (1, 0)]) == ERROR               # undeclared child
    assert orc.tree_state([(0, 1), (2, 0)]) == WAITING             # gen 1 not there yet
    assert orc.tree_state([(0, 1), (1, 0), (2, 0)]) == ERROR       # gen 2 never declared
    # a list: one tile per generation, back to front
    lst = [(0, 1), (1, 1), (2, 1), (3, 0)]
    assert orc.tree_progress(lst) == (COMPLETE, 3, 0)
    assert orc.tree_progress(lst[:3]) == (WAITING, 3, 1)


@pytest.mark.parametrize("seed", range(40))
def test_oracle_tree_constructed(seed):
    """Built trees: every proper prefix of any arrival order waits, the whole
    set completes; one tile less waits; one tile more is an error."""
    rng = random.Random(seed)
    nodes = random_tree(rng)
    for _ in range(5):
        perm = nodes[:]
        rng.shuffle(perm)
        trace = orc.tree_trace(perm)
        assert trace[-1] == COMPLETE
        assert all(s == WAITING for s in trace[:-1])
    drop = rng.randrange(len(nodes))
    assert orc.tree_state(nodes[:drop] + nodes[drop + 1:]) == WAITING
    max_gen = max(g for g, _ in nodes)
    extra = (rng.randint(0, max_gen + 1), rng.randint(0, 2))
    assert orc.tree_state(nodes + [extra]) == ERROR


# ------------------------------------------------------------ library tracker
def mutate(rng, nodes):
    """A sequence of arrivals that may or may not form a valid tree."""
    out = nodes[:]
    r = rng.random()
    if r < 0.25 and len(out) > 1:
        out.pop(rng.randrange(1, len(out)))
    elif r < 0.5:
        out.insert(rng.randrange(len(out) + 1), (rng.randint(0, 4), rng.randint(0, 2)))
    elif r < 0.75 and len(out) > 1:
        i = rng.randrange(len(out))
        out[i] = (out[i][0], max(0, out[i][1] + rng.choice((-1, 1))))
    rng.shuffle(out)
    return out


@pytest.mark.parametrize("seed", range(12))
def test_tracker_matches_oracle(dfb_host, seed):
    import paper_2305_07083_amd as dfb
    rng = random.Random(1000 + seed)
    n_tiles = 16
    seqs = [mutate(rng, random_tree(rng)) if rng.random() < 0.7 else random_tree(rng) for _ in range(n_tiles)]
    for s in seqs:
        if rng.random() < 0.5:
            rng.shuffle(s)
    # interleave the tiles' arrivals
    events = [(t, i) for t in range(n_tiles) for i in range(len(seqs[t]))]
    pos = [0] * n_tiles
    order = []
    for t, _ in events:
        order.append(t)
    rng.shuffle(order)
    with dfb.Tree(n_tiles) as tree:
        for t in order:
            g, c = seqs[t][pos[t]]
            pos[t] += 1
            before = orc.tree_state(seqs[t][:pos[t] - 1]) if pos[t] > 1 else WAITING
            st, done = tree.add(t, g, c)
            want = orc.tree_progress(seqs[t][:pos[t]])
            if want[0] == ERROR:
                assert st == dfb.DFB_ERR_TREE
                assert not done
                assert tree.query(t)[0] == -1
            else:
                assert st == dfb.DFB_OK
                assert done == (want[0] == COMPLETE and before != COMPLETE)
                state, gen, missing = tree.query(t)
                assert (state, gen, missing) == ({COMPLETE: 1, WAITING: 0}[want[0]], want[1], want[2])
        tree.new_frame()
        for t in range(n_tiles):
            assert tree.query(t) == (0, 0, 1)


def test_tracker_argument_errors(dfb_host):
    import paper_2305_07083_amd as dfb
    with dfb.Tree(2) as tree:
        assert tree.add(2, 0, 0)[0] == dfb.DFB_ERR_INVALID_ARG
        assert tree.add(-1, 0, 0)[0] == dfb.DFB_ERR_INVALID_ARG
        assert tree.add(0, -1, 0)[0] == dfb.DFB_ERR_INVALID_ARG
        assert tree.add(0, 65536, 0)[0] == dfb.DFB_ERR_INVALID_ARG
        assert tree.add(0, 0, -1)[0] == dfb.DFB_ERR_INVALID_ARG
        assert tree.query(0) == (0, 0, 1)           # rejected arrivals change nothing
        assert tree.add(0, 0, 1) == (dfb.DFB_OK, False)
        assert tree.add(0, 65535, 0) == (dfb.DFB_OK, False)   # far generation: counted, undecided
        assert tree.add(0, 1, 0) == (dfb.DFB_ERR_TREE, False)  # completes gen 1, gen 65535 is extra
        assert tree.add(1, 0, 0) == (dfb.DFB_OK, True)
        assert tree.add(1, 1, 0) == (dfb.DFB_ERR_TREE, False)  # after completion


# ------------------------------------------------------------ sample assignment
def test_oracle_assign_uniform_and_sum():
    assert orc.assign_samples([np.inf] * 4, 10) == [3, 3, 2, 2]
    assert orc.assign_samples([0.0, 0.0, 0.0], 4) == [2, 1, 1]
    assert orc.assign_samples([np.nan, -1.0], 3) == [2, 1]
    assert orc.assign_samples([1.0, 1.0, 1.0], 4) == [2, 1, 1]   # equal remainders: smaller id first
    assert orc.assign_samples([0.0, 2.0, 0.0, 6.0], 8) == [0, 2, 0, 6]
    assert orc.assign_samples([1.0, 2.0], 0) == [0, 0]


@pytest.mark.parametrize("seed", range(30))
def test_oracle_assign_brute_force(seed):
    """Hamilton's apportionment is the integer split of `extra` closest to the
    quotas in the squared sense; each share is a quota rounded down or up."""
    rng = np.random.default_rng(seed)
    T = int(rng.integers(1, 5))
    E = int(rng.integers(0, 8))
    v = rng.random(T).astype(np.float32)
    v[rng.random(T) < 0.2] = 0.0
    c = orc.assign_samples(v, E)
    assert sum(c) == E
    w = np.where(np.isfinite(v) & (v > 0), v.astype(np.float64), 0.0)
    if w.sum() == 0:
        return
    q = E * w / w.sum()
    assert all(math.floor(qi) <= ci <= math.ceil(qi) for qi, ci in zip(q, c))
    best = min(sum((a - b) ** 2 for a, b in zip(comp, q))
               for comp in itertools.product(range(E + 1), repeat=T) if sum(comp) == E)
    assert sum((a - b) ** 2 for a, b in zip(c, q)) <= best + 1e-9


def test_oracle_assign_scale_invariant():
    rng = np.random.default_rng(7)
    v = rng.random(100).astype(np.float32)
    assert orc.assign_samples(v, 1234) == orc.assign_samples(v * np.float32(4.0), 1234)


@pytest.mark.parametrize("seed", range(8))
def test_library_assign_matches_oracle(dfb_host, seed):
    import paper_2305_07083_amd as dfb
    rng = np.random.default_rng(100 + seed)
    T = int(rng.integers(1, 3000))
    v = (rng.random(T) ** 3).astype(np.float32)
    kind = seed % 4
    if kind == 1:
        v[rng.random(T) < 0.3] = 0.0
        v[rng.random(T) < 0.05] = np.nan
        v[rng.random(T) < 0.05] = np.inf
    elif kind == 2:
        v = np.round(v * 4).astype(np.float32)  # many equal values: ties
    elif kind == 3:
        v[:] = np.inf
    for extra in (0, 1, T - 1, T, 3 * T + 7, int(rng.integers(0, 100000))):
        got = dfb.dfb_assign_samples_host(v, extra)
        assert got.tolist() == orc.assign_samples(v, extra), (kind, extra)


def test_library_assign_errors(dfb_host):
    import paper_2305_07083_amd as dfb
    with pytest.raises(dfb.DfbError):
        dfb.dfb_assign_samples_host(np.ones(3, np.float32), -1)
    with pytest.raises(dfb.DfbError):
        dfb.dfb_assign_samples_host(np.ones(3, np.float32), 2 ** 31)
    with pytest.raises(dfb.DfbError):
        dfb.dfb_assign_samples_host(np.ones(0, np.float32), 1)
