"""Pins of the FP64 oracle against what the paper and the mathematics fix.

None of these compares the oracle with itself: each checks a printed value of
the paper, a closed form worked by hand, a theorem of the paper, or a brute
force enumeration.  The mutation tests (test_oracle_mutants.py) plant
plausible mistakes in a copy of the oracle and require one of these to fail.
"""
import itertools

import numpy as np
import pytest

import oracle
from paper_2004_08227_amd import workloads as W
from tests.golden.fixtures import read_kv

GOLD = read_kv("prop3_counterexample.txt")


# --------------------------------------------------------------------------
# (H) on the worked example printed in Appendix B (proof of Proposition 3).
# --------------------------------------------------------------------------

@pytest.mark.parametrize("case", ["case1", "case2"])
def test_handshake_matches_paper_worked_example(case):
    T = GOLD["theta_uv"]
    Te, hu, hv = oracle.update("H", T, GOLD[f"{case}.theta_u"], GOLD[f"{case}.theta_v"])
    # dyadic numbers: the paper's values are exact in binary floating point
    assert np.array_equal(hu, GOLD[f"{case}.H_u"])
    assert np.array_equal(hv, GOLD[f"{case}.H_v"])
    # new pairwise = g - H_u - H_v; g = theta_uv + theta_u + theta_v
    g = T + GOLD[f"{case}.theta_u"][:, None] + GOLD[f"{case}.theta_v"][None, :]
    assert np.array_equal(Te, g - hu[:, None] - hv[None, :])


def test_worked_example_fixes_the_orientation():
    """Processing the same edge with u and v swapped (the table transposed)
    does not give the printed values of the second case (it gives u = (0,
    4.5), v = (0, 0.5) instead of (0, 4), (0, 1)): the fixture pins which
    node gets the first correction.  (The first case happens to give the same
    numbers in both orientations.)"""
    T = GOLD["theta_uv"]
    _, hv_sw, hu_sw = oracle.update("H", T.T, GOLD["case2.theta_v"], GOLD["case2.theta_u"])
    assert np.array_equal(hu_sw, [0.0, 4.5]) and np.array_equal(hv_sw, [0.0, 0.5])
    assert not np.array_equal(hu_sw, GOLD["case2.H_u"])


def test_mplp_and_uniform_closed_form_on_worked_example():
    """(M) and (U) of Sec. 4 on the worked example, worked by hand:
    g = [[0+4+2, 1+4+0], [7+0+2, 5+0+0]] = [[6, 5], [9, 5]];
    (M): u gets half the row minima (5/2, 5/2), v half the column minima
    (6/2, 5/2); (U): both get half the overall minimum 5/2."""
    T = GOLD["theta_uv"]
    _, mu, mv = oracle.update("M", T, GOLD["case1.theta_u"], GOLD["case1.theta_v"])
    assert np.array_equal(mu, [2.5, 2.5]) and np.array_equal(mv, [3.0, 2.5])
    _, uu, uv = oracle.update("U", T, GOLD["case1.theta_u"], GOLD["case1.theta_v"])
    assert np.array_equal(uu, [2.5, 2.5]) and np.array_equal(uv, [2.5, 2.5])
    # second case: g = theta_uv = [[0, 1], [7, 5]] -> (M): (0, 5/2), (0, 1/2)
    _, mu, mv = oracle.update("M", T, GOLD["case2.theta_u"], GOLD["case2.theta_v"])
    assert np.array_equal(mu, [0.0, 2.5]) and np.array_equal(mv, [0.0, 0.5])


# --------------------------------------------------------------------------
# Per-edge properties (Sec. 4, Prop. 1, Def. 1, Prop. 2).
# --------------------------------------------------------------------------

def _random_edge(rng, L):
    return rng.normal(size=(L, L)), rng.normal(size=L), rng.normal(size=L)


@pytest.mark.parametrize("L", [1, 2, 3, 5, 8, 13])
def test_update_postconditions(L):
    rng = np.random.default_rng(100 + L)
    for _ in range(40):
        T, a, b = _random_edge(rng, L)
        g = T + a[:, None] + b[None, :]
        for rule in "HMU":
            Te, hu, hv = oracle.update(rule, T, a, b)
            tol = 1e-12 * (1 + np.abs(g).max())
            # reparametrization: the aggregated cost is unchanged (Sec. 4)
            assert np.allclose(Te + hu[:, None] + hv[None, :], g, rtol=0, atol=tol)
            # restricted dual attains its maximum min g (Eq. 4 and Prop. 1)
            assert abs(hu.min() + hv.min() + Te.min() - g.min()) <= 4 * tol
            # Def. 1 normalization: min of the new pairwise is 0
            assert abs(Te.min()) <= 4 * tol
            # Prop. 1: a label pair minimal for u, v and the edge at once
            su = np.flatnonzero(hu <= hu.min() + 4 * tol)
            sv = np.flatnonzero(hv <= hv.min() + 4 * tol)
            assert (Te[np.ix_(su, sv)] <= 4 * tol).any()
            if rule == "H":
                # (H) leaves zero row and column minima (Sec. 4, after (H))
                assert np.abs(Te.min(axis=1)).max() <= 4 * tol
                assert np.abs(Te.min(axis=0)).max() <= 4 * tol


@pytest.mark.parametrize("L", [1, 2, 4, 7])
def test_update_dominance_H_ge_M_ge_U(L):
    """Prop. 2: component-wise H >= M >= U for any aggregated cost."""
    rng = np.random.default_rng(7 + L)
    for _ in range(60):
        T, a, b = _random_edge(rng, L)
        _, hu, hv = oracle.update("H", T, a, b)
        _, mu, mv = oracle.update("M", T, a, b)
        _, uu, uv = oracle.update("U", T, a, b)
        assert (hu >= mu - 1e-12).all() and (hv >= mv - 1e-12).all()
        assert (mu >= uu - 1e-12).all() and (mv >= uv - 1e-12).all()


# --------------------------------------------------------------------------
# Dual bound, energy, decode, brute force: hand-worked small cases.
# --------------------------------------------------------------------------

def _hand_model():
    """n=3 path 0-1-2 plus edge 0-2, L=2; numbers chosen for hand work."""
    edges = np.array([[0, 1], [1, 2], [0, 2]], dtype=np.int32)
    un = np.array([[1.0, 0.0], [0.0, 2.0], [3.0, 1.0]])
    pw = np.array([
        [[0.0, 4.0], [1.0, 2.0]],     # (0,1): rows label of 0, cols label of 1
        [[2.0, 0.0], [5.0, 1.0]],     # (1,2)
        [[1.0, 3.0], [0.0, 6.0]],     # (0,2)
    ])
    return W.Model(3, 2, edges, un, pw)


def test_energy_and_initial_dual_by_hand():
    m = _hand_model()
    st = oracle.State(m)
    # Eq. (1) for y = (1, 0, 1): unaries 0 + 0 + 1, pairwise (1,0)->1, (0,1)->0, (1,1)->6 => 8
    assert st.energy(np.array([1, 0, 1], np.int32)) == 8.0
    # Eq. (3) at phi = 0: node minima 0 + 0 + 1, edge minima 0 + 0 + 0 => 1
    assert st.dual() == 1.0
    # brute force agrees with the energy of every labelling
    table = {}
    for y in itertools.product(range(2), repeat=3):
        table[y] = st.energy(np.array(y, np.int32))
    best = min(table.values())
    e, lab = oracle.bruteforce(m)
    assert e == best and table[tuple(lab)] == best
    # the hand enumeration: y=(1,0,0): 0+0+3 + 1+2+0 = 6; (1,0,1): 8; (0,0,0): 1+0+3+0+2+1 = 7;
    # (0,0,1): 1+0+1+0+0+3 = 5; (1,1,0): 0+2+3+2+5+0 = 12; (1,1,1): 0+2+1+2+1+6 = 12;
    # (0,1,0): 1+2+3+4+5+1 = 16; (0,1,1): 1+2+1+4+1+3 = 12  => MAP 5 at (0,0,1)
    assert e == 5.0 and list(lab) == [0, 0, 1]


def test_decode_by_hand():
    """Eq. (5) on the input costs (phi = 0): node 0 takes argmin of its unary
    (1, 0) -> 1; node 1 adds column of edge (0,1) at row 1: (0,2)+(1,2) =
    (1, 4) -> 0; node 2 adds edge (1,2) row 0 and edge (0,2) row 1:
    (3,1) + (2,0) + (0,6) = (5, 7) -> 0."""
    st = oracle.State(_hand_model())
    assert list(st.decode()) == [1, 0, 0]


def test_initial_dual_counts_edge_minima_by_hand():
    """Eq. (3) at phi = 0 for n=2, L=2: min(1, 2) + min(0, 3) +
    min(2, 5, 4, 3) = 1 + 0 + 2 = 3."""
    m = W.Model(2, 2, np.array([[0, 1]], np.int32), np.array([[1.0, 2.0], [0.0, 3.0]]),
                np.array([[[2.0, 5.0], [4.0, 3.0]]]))
    assert oracle.State(m).dual() == 3.0


def test_decode_reads_rows_of_the_lower_node():
    """Eq. (5) with the table row given by the earlier node's label: node 0
    takes label 0 (unary (0, 1)); node 1 adds row 0 of [[1, 2], [0, 9]],
    (1, 2) -> label 0.  Reading the column instead would give (1, 0) -> 1."""
    m = W.Model(2, 2, np.array([[0, 1]], np.int32), np.array([[0.0, 1.0], [0.0, 0.0]]),
                np.array([[[1.0, 2.0], [0.0, 9.0]]]))
    assert list(oracle.State(m).decode()) == [0, 0]


def test_decode_ties_go_to_lowest_label():
    m = W.Model(2, 3, np.array([[0, 1]], np.int32), np.zeros((2, 3)), np.zeros((1, 3, 3)))
    assert list(oracle.State(m).decode()) == [0, 0]


def test_single_edge_one_update_reaches_map():
    """One edge: one block-optimal update maximizes the whole dual, which then
    equals the MAP energy min g (Prop. 1 with Eq. (3) <= Eq. (1))."""
    for L in (1, 2, 3, 6):
        for seed in range(5):
            rng = np.random.default_rng(seed)
            m = W.Model(2, L, np.array([[0, 1]], np.int32), rng.random((2, L)), rng.random((1, L, L)))
            st, tr = oracle.run_model(m, 1)
            e, _ = oracle.bruteforce(m)
            assert abs(tr[0] - e) <= 1e-12


def test_zero_pairwise_dual_is_map():
    rng = np.random.default_rng(3)
    n, L = 6, 3
    edges = W.complete_edges(n)
    m = W.Model(n, L, edges, rng.random((n, L)), np.zeros((edges.shape[0], L, L)))
    st, tr = oracle.run_model(m, 5)
    target = m.unaries.min(axis=1).sum()
    assert np.all(np.abs(tr - target) <= 1e-12)
    assert list(st.decode()) == list(m.unaries.argmin(axis=1))


# --------------------------------------------------------------------------
# Whole-iteration properties (Sec. 5, App. B).
# --------------------------------------------------------------------------

@pytest.mark.parametrize("seed", range(4))
def test_dual_monotone_and_below_map_and_energy_invariant(seed):
    m = W.tiny(seed, n=6, L=3)
    e_map, _ = oracle.bruteforce(m)
    for rule in "HMU":
        st, tr = oracle.run_model(m, 60, rule=rule)
        d0 = oracle.State(m).dual()
        full = np.concatenate([[d0], tr])
        assert np.all(np.diff(full) >= -1e-12), rule        # monotone (App. B lemma)
        assert full.max() <= e_map + 1e-12, rule            # D <= E(y) (Eq. 3)
        lab = st.decode()
        assert st.energy(lab) >= e_map - 1e-12
        rng = np.random.default_rng(seed)
        for _ in range(20):                                  # E(y|theta^phi) = E(y|theta)
            y = rng.integers(0, m.L, m.n).astype(np.int32)
            assert abs(st.energy(y, reparametrized=True) - st.energy(y)) <= 1e-11


def test_dual_monotone_after_every_single_update():
    m = W.tiny(11, n=5, L=3)
    st = oracle.State(m)
    d = st.dual()
    for _ in range(3):
        for k in range(st.n_steps):
            for e in st.order[st.step_ptr[k]:st.step_ptr[k + 1]]:
                u, v = st.edges[e]
                Te, hu, hv = oracle.update("H", st.Te[e], st.Tu[u], st.Tu[v])
                st.Te[e], st.Tu[u], st.Tu[v] = Te, hu, hv
                d2 = st.dual()
                assert d2 >= d - 1e-12
                d = d2


def test_tiny_k8_l4_200_iterations_below_bruteforce_map():
    m = W.tiny(0)
    st, tr = oracle.run_model(m, 200)
    e_map, _ = oracle.bruteforce(m)
    assert np.all(np.diff(tr) >= -1e-12)
    assert tr[-1] <= e_map + 1e-12
    assert st.energy(st.decode()) >= e_map - 1e-12


@pytest.mark.parametrize("seed", range(4))
def test_iteration_dominance_H_over_M_over_U(seed):
    """Thm. 2: from the same start and edge order, one (H) iteration gives a
    dual at least that of one (M) iteration, which dominates (U)."""
    m = W.tiny(seed, n=7, L=3)
    for warm in (0, 3):
        base = oracle.State(m)
        base.run(warm, rule="M")
        ds = {}
        for rule in "HMU":
            st = oracle.State(m)
            st.Tu[:] = base.Tu
            st.Te[:] = base.Te
            st.run(1, rule=rule)
            ds[rule] = st.dual()
        assert ds["H"] >= ds["M"] - 1e-12 and ds["M"] >= ds["U"] - 1e-12


@pytest.mark.parametrize("seed", range(3))
def test_trees_reach_the_map(seed):
    """The LP relaxation is tight on trees and MPLP++ converges to node-edge
    agreement (Thm. 1), so the dual reaches the MAP energy on a chain."""
    m = W.chain(7, 3, seed)
    st, tr = oracle.run_model(m, 200)
    e_map, _ = oracle.bruteforce(m)
    assert abs(tr[-1] - e_map) <= 1e-9


@pytest.mark.parametrize("seed", range(3))
def test_submodular_binary_reaches_the_map(seed):
    """BCA solves submodular problems exactly (Sec. 2)."""
    rng = np.random.default_rng(seed)
    n = 6
    e = W.complete_edges(n)
    pw = rng.random((e.shape[0], 2, 2))
    d = pw[:, 0, 0] + pw[:, 1, 1] - pw[:, 0, 1] - pw[:, 1, 0]
    pw[:, 1, 1] -= np.maximum(d, 0) + 0.1
    m = W.Model(n, 2, e, rng.random((n, 2)), pw)
    st, tr = oracle.run_model(m, 200)
    e_map, _ = oracle.bruteforce(m)
    assert abs(tr[-1] - e_map) <= 1e-9


def test_edges_of_a_matching_commute():
    """Sec. 6: edges of one matching share no node, so their order inside the
    matching does not change the result (bitwise)."""
    m = W.tiny(5, n=9, L=3)
    a = oracle.State(m)
    a.run(7)
    rng = np.random.default_rng(0)
    order = a.order.copy()
    for k in range(a.n_steps):
        lo, hi = a.step_ptr[k], a.step_ptr[k + 1]
        order[lo:hi] = rng.permutation(order[lo:hi])
    b = oracle.State(m, step_ptr=a.step_ptr, order=order)
    b.run(7)
    assert np.array_equal(a.Tu, b.Tu) and np.array_equal(a.Te, b.Te)


@pytest.mark.parametrize("rule", ["H", "M", "U"])
def test_dual_moves_by_a_constant_added_to_one_node_or_edge(rule):
    """Adding c to every label of one node's unary, or to every entry of one
    edge's table, adds c to the energy of every labelling; every update
    (Sec. 4) passes such a uniform shift through without moving an argmin,
    so the dual after K iterations moves by exactly c (up to the rounding of
    the sums).  A dropped or doubled half in an update breaks this."""
    m = W.uniform(7, 5, seed=11, dtype=np.float64)
    c = 0.375
    d0 = oracle.dual_after(m, 3, rule=rule)
    for u in range(m.n):
        du = np.zeros_like(m.unaries)
        du[u] = c
        mu = W.Model(m.n, m.L, m.edges, m.unaries + du, m.pairwise)
        assert abs(oracle.dual_after(mu, 3, rule=rule) - (d0 + c)) <= 1e-12 * max(1.0, abs(d0))
    for e in range(0, m.m, 4):
        dp = np.zeros_like(m.pairwise)
        dp[e] = c
        me = W.Model(m.n, m.L, m.edges, m.unaries, m.pairwise + dp)
        assert abs(oracle.dual_after(me, 3, rule=rule) - (d0 + c)) <= 1e-12 * max(1.0, abs(d0))


def test_threads_do_not_change_results():
    m = W.uniform(24, 5, seed=2, dtype=np.float64)
    a = oracle.State(m)
    b = oracle.State(m)
    ta = a.run(5, trace=True, nthreads=1)
    tb = b.run(5, trace=True, nthreads=4)
    assert np.array_equal(a.Tu, b.Tu) and np.array_equal(a.Te, b.Te) and np.array_equal(ta, tb)


def test_reversed_edge_input_is_transposed():
    m = W.tiny(2, n=5, L=3)
    flip = W.Model(m.n, m.L, m.edges[:, ::-1].copy(), m.unaries, np.transpose(m.pairwise, (0, 2, 1)).copy())
    a, ta = oracle.run_model(m, 5)
    b, tb = oracle.run_model(flip, 5)
    assert np.array_equal(ta, tb) and np.array_equal(a.Tu, b.Tu)


@pytest.mark.parametrize("bad", ["self", "range", "dup", "nan"])
def test_invalid_models_rejected(bad):
    m = W.tiny(0, n=4, L=2)
    edges, un, pw = m.edges.copy(), m.unaries.copy(), m.pairwise.copy()
    if bad == "self":
        edges[0] = [1, 1]
    elif bad == "range":
        edges[0] = [0, 9]
    elif bad == "dup":
        edges[1] = edges[0][::-1]
    else:
        pw[0, 0, 0] = np.nan
    with pytest.raises(oracle.OracleError):
        oracle.State(W.Model(m.n, m.L, edges, un, pw))
