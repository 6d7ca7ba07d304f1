"""Pins of the oracle's edge schedule (Sec. 6, Alg. 1) against the
definitions: every queue entry is a matching, the queue covers every edge
exactly once, complete graphs get the optimal number of rounds, and a greedy
round is a maximal matching of the edges left."""
import numpy as np
import pytest

import oracle
from paper_2004_08227_amd import workloads as W


def check_schedule(n, edges, step_ptr, order):
    m = edges.shape[0]
    assert step_ptr[0] == 0 and step_ptr[-1] == m
    assert np.all(np.diff(step_ptr) > 0)
    assert sorted(order.tolist()) == list(range(m))           # each edge once
    for k in range(len(step_ptr) - 1):
        es = order[step_ptr[k]:step_ptr[k + 1]]
        nodes = edges[es].ravel()
        assert len(set(nodes.tolist())) == nodes.size           # a matching
        keys = edges[es, 0].astype(np.int64) * n + edges[es, 1]
        assert np.all(np.diff(keys) > 0)                        # ascending (u, v)


@pytest.mark.parametrize("n", [1, 2, 3, 4, 5, 6, 7, 8, 9, 16, 33, 200])
def test_complete_graph_rounds(n):
    edges = W.complete_edges(n)
    sp, order = oracle.schedule(n, edges)
    if n == 1:
        assert len(sp) == 1
        return
    check_schedule(n, edges, sp, order)
    S = len(sp) - 1
    # a K_n needs at least n-1 rounds (n even) or n rounds (n odd): each
    # node meets n-1 edges, at most one per round; each round of an odd
    # graph leaves a node out.  The circle method attains both bounds.
    assert S == (n - 1 if n % 2 == 0 else n)
    sizes = np.diff(sp)
    assert np.all(sizes == n // 2)


@pytest.mark.parametrize("seed,n,p", [(0, 10, 0.3), (1, 30, 0.1), (2, 50, 0.5), (3, 12, 0.9), (4, 40, 0.05)])
def test_greedy_rounds_are_maximal_matchings(seed, n, p):
    m = W.random_graph_model(n, 2, p, seed=seed)
    edges = m.edges
    if edges.shape[0] == 0:
        return
    sp, order = oracle.schedule(n, edges)
    check_schedule(n, edges, sp, order)
    remaining = set(range(edges.shape[0]))
    for k in range(len(sp) - 1):
        es = set(order[sp[k]:sp[k + 1]].tolist())
        busy = set(edges[list(es)].ravel().tolist())
        remaining -= es
        for e in remaining:                  # nothing left could be added
            u, v = edges[e]
            assert u in busy or v in busy
    # lower bound: at least the maximum degree many rounds
    deg = np.bincount(edges.ravel(), minlength=n)
    assert len(sp) - 1 >= deg.max()


def test_greedy_first_round_by_hand():
    """Path 0-1-2-3 plus chord 0-2: scanning (0,1), (0,2), (1,2), (2,3)
    greedily gives rounds {(0,1), (2,3)}, {(0,2)}, {(1,2)}."""
    edges = np.array([[0, 1], [1, 2], [2, 3], [0, 2]], np.int32)
    sp, order = oracle.schedule(4, edges)
    rounds = [sorted(tuple(edges[e]) for e in order[sp[k]:sp[k + 1]]) for k in range(len(sp) - 1)]
    assert rounds == [[(0, 1), (2, 3)], [(0, 2)], [(1, 2)]]


def test_circle_method_first_rounds_by_hand():
    """K_4 by the round-robin rule: round r pairs 3 with r and (r+1) with
    (r-1) mod 3: {(0,3), (1,2)}, {(1,3), (0,2)}, {(2,3), (0,1)}."""
    edges = W.complete_edges(4)
    sp, order = oracle.schedule(4, edges)
    rounds = [sorted(tuple(int(x) for x in edges[e]) for e in order[sp[k]:sp[k + 1]]) for k in range(3)]
    assert rounds == [[(0, 3), (1, 2)], [(0, 2), (1, 3)], [(0, 1), (2, 3)]]
