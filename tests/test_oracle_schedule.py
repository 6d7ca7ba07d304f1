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


# ---- the edge-colouring schedule (Delta + 1 matchings) ----

@pytest.mark.parametrize("seed,n,p", [(0, 10, 0.3), (1, 30, 0.1), (2, 50, 0.5), (3, 12, 0.9), (4, 40, 0.05),
                                      (5, 120, 0.2), (6, 7, 0.6)])
def test_colour_schedule_is_a_proper_colouring_within_vizing(seed, n, p):
    m = W.random_graph_model(n, 2, p, seed=seed)
    edges = m.edges
    if edges.shape[0] == 0:
        return
    sp, order = oracle.schedule(n, edges, "color")
    check_schedule(n, edges, sp, order)
    deg = np.bincount(edges.ravel(), minlength=n)
    S = len(sp) - 1
    if edges.shape[0] < n * (n - 1) // 2:
        assert deg.max() <= S <= deg.max() + 1      # Vizing: Delta or Delta + 1 colours


def test_colour_schedule_class_two_graphs_need_delta_plus_one():
    """The odd cycle C_5 (Delta = 2) and the Petersen graph (Delta = 3) have no
    Delta-edge-colouring, so a proper colouring uses exactly Delta + 1."""
    c5 = np.array([[i, (i + 1) % 5] for i in range(5)], np.int32)
    c5 = np.sort(c5, axis=1)
    sp, order = oracle.schedule(5, c5, "color")
    check_schedule(5, c5, sp, order)
    assert len(sp) - 1 == 3
    outer = [(i, (i + 1) % 5) for i in range(5)]
    spokes = [(i, i + 5) for i in range(5)]
    inner = [(5 + i, 5 + (i + 2) % 5) for i in range(5)]
    pet = np.sort(np.array(outer + spokes + inner, np.int32), axis=1)
    sp, order = oracle.schedule(10, pet, "color")
    check_schedule(10, pet, sp, order)
    assert len(sp) - 1 == 4


def test_colour_schedule_star_and_path():
    """A star K_{1,k} needs k colours (all edges meet) and gets k.  A path
    could do with 2 but the rule, which guarantees only Delta + 1, gives 3:
    (0,1) takes 0; (1,2): fan [2, 0], c = d = 1, so 1; (2,3): fan [3, 1]
    (colour 1 of 2-1 is free at 3), c = 0 free at 2, d = 2 free at 1, no
    d-path at 2, w = 3, so 2; the pattern repeats."""
    k = 9
    star = np.array([[0, i] for i in range(1, k + 1)], np.int32)
    sp, order = oracle.schedule(k + 1, star, "color")
    check_schedule(k + 1, star, sp, order)
    assert len(sp) - 1 == k
    path = np.array([[i, i + 1] for i in range(12)], np.int32)
    sp, order = oracle.schedule(13, path, "color")
    check_schedule(13, path, sp, order)
    assert len(sp) - 1 == 3
    assert [int(e) for e in order[sp[0]:sp[1]]] == [0, 3, 6, 9]


def test_colour_schedule_by_hand():
    """Triangle 0-1-2 with pendant 2-3, coloured in (u, v) order with the
    fixed choices of the rule:
      (0,1): fan [1], c = d = 0 -> colour 0;
      (0,2): fan [2, 1] (edge 0-1 has colour 0, free at 2), c = d = 1, w = 2
             -> colour 1;
      (1,2): fan [2, 0], c = 1 free at 1, d = 2 free at 0; no d-path at 1;
             w = 2 (2 free there) -> colour 2;
      (2,3): fan [3, 0, 1] (colour 1 of 2-0 is free at 3, colour 2 of 2-1
             at 0), c = 0 free at 2, d = 1 free at 1; the path 2-0 (1),
             0-1 (0) swaps to 2-0 = 0, 0-1 = 1; w = 3 -> colour 1.
    Colour classes: {(0,2)}, {(0,1), (2,3)}, {(1,2)}."""
    edges = np.array([[0, 1], [0, 2], [1, 2], [2, 3]], np.int32)
    sp, order = oracle.schedule(4, edges, "color")
    rounds = [sorted(tuple(int(x) for x in edges[e]) for e in order[sp[k]:sp[k + 1]]) for k in range(len(sp) - 1)]
    assert rounds == [[(0, 2)], [(0, 1), (2, 3)], [(1, 2)]]


def test_colour_schedule_of_a_complete_graph_is_the_round_robin():
    edges = W.complete_edges(10)
    sp_c, o_c = oracle.schedule(10, edges, "color")
    sp_g, o_g = oracle.schedule(10, edges, "greedy")
    assert np.array_equal(sp_c, sp_g) and np.array_equal(o_c, o_g)
