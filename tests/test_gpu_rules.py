"""GPU tests of the other BCA-updates of Sec. 4: MPLP (M) and uniform (U),
on the per-matching engine (and on the mailbox engine, bitwise the
per-matching one), against the paper's two-node example (printed
values and the closed forms of (M) and (U) on the same inputs), the FP64
oracle (1e-12 in FP64, 1e-5 in FP32), and the dominance of one (H)
iteration over (M) over (U) from the same start (Sec. 5)."""
import numpy as np
import pytest

import oracle
from paper_2004_08227_amd import workloads as W

pytestmark = pytest.mark.gpu
M = pytest.importorskip("paper_2004_08227_amd")


def _announce(*a):
    print("CASE", *a, flush=True)


def _rel(a, b):
    return abs(a - b) / max(1.0, abs(b))


def _two_node(dtype):
    # the worked example of the paper: theta_uv = [[0, 1], [7, 5]], unaries
    # theta_u = (4, 0), theta_v = (2, 0), zero messages
    return W.Model(2, 2, np.array([[0, 1]], np.int32), np.array([[4.0, 0.0], [2.0, 0.0]], dtype),
                   np.array([[[0.0, 1.0], [7.0, 5.0]]], dtype), "two_node")


@pytest.mark.parametrize("dtype", [np.float64, np.float32])
@pytest.mark.parametrize("rule,u,v", [("H", (2.5, 2.5), (3.5, 2.5)),   # printed in the paper
                                      ("M", (2.5, 2.5), (3.0, 2.5)),   # (M): halves of the row / column minima
                                      ("U", (2.5, 2.5), (2.5, 2.5))])  # (U): half of min g = 5
def test_two_node_example(rule, u, v, dtype):
    _announce("two node", rule, dtype.__name__)
    model = _two_node(dtype)
    with M.Solver.from_model(model) as s:
        s.set_option(M.OPT_RULE, {"H": M.RULE_H, "M": M.RULE_M, "U": M.RULE_U}[rule])
        s.iterate(1)
        U, phi = s.get_state()
        d = s.dual_bound()
    assert np.array_equal(U[0], np.array(u, U.dtype)), U
    assert np.array_equal(U[1], np.array(v, U.dtype)), U
    # every update here leaves min of the reparametrized pairwise at 0, so
    # the dual is the sum of the unary minima; (H) and (M) reach min g = 5
    assert d == min(u) + min(v)


def _f64(model):
    return W.Model(model.n, model.L, model.edges, model.unaries.astype(np.float64),
                   model.pairwise.astype(np.float64), model.name + "_f64")


CASES = [
    ("tiny", lambda: W.tiny(0), 30),
    ("pose_ragged", lambda: W.pose(21, 13, seed=4), 10),
    ("uniform_L32", lambda: W.uniform(16, 32, seed=6), 10),
    ("potts_er", lambda: W.potts_er(50, 16, 0.3, seed=7), 10),
    ("uniform_L65", lambda: W.uniform(9, 65, seed=10), 5),
]


@pytest.mark.parametrize("rule", ["M", "U"])
@pytest.mark.parametrize("name,make,iters", CASES, ids=[c[0] for c in CASES])
def test_rule_fp64_matches_oracle(name, make, iters, rule):
    _announce("fp64", name, rule)
    model = _f64(make())
    st, ref = oracle.run_model(model, iters, rule=rule)
    with M.Solver.from_model(model) as s:
        s.set_option(M.OPT_RULE, M.RULE_M if rule == "M" else M.RULE_U)
        assert s.info("engine") == M.ENGINE_STEP
        tr = s.iterate_trace(iters)
        d = s.dual_bound()
        U, phi = s.get_state()
    assert np.max(np.abs(tr - ref) / np.maximum(1.0, np.abs(ref))) <= 1e-12
    assert _rel(d, st.dual()) <= 1e-12
    assert np.max(np.abs(U - st.Tu)) <= 1e-12 * max(1.0, np.abs(st.Tu).max())
    Te = st.pairwise - phi[:, 0, :, None] - phi[:, 1, None, :]
    assert np.max(np.abs(Te - st.Te)) <= 1e-12 * max(1.0, np.abs(st.Te).max())


@pytest.mark.parametrize("rule", ["M", "U"])
@pytest.mark.parametrize("name,make,iters", [("pose", lambda: W.pose(40, 64, seed=3), 20),
                                             ("uniform_L32", lambda: W.uniform(30, 32, seed=6), 20),
                                             ("potts_er", lambda: W.potts_er(80, 16, 0.3, seed=7), 20)],
                         ids=["pose", "uniform_L32", "potts_er"])
def test_rule_fp32_matches_oracle(name, make, iters, rule):
    _announce("fp32", name, rule)
    model = make()
    st, ref = oracle.run_model(model, iters, rule=rule)
    with M.Solver.from_model(model) as s:
        s.set_option(M.OPT_RULE, M.RULE_M if rule == "M" else M.RULE_U)
        tr = s.iterate_trace(iters)
        d = s.dual_bound()
    assert np.max(np.abs(tr - ref) / np.maximum(1.0, np.abs(ref))) <= 1e-5
    assert _rel(d, ref[-1]) <= 1e-5


@pytest.mark.parametrize("name,make,iters", CASES[1:] + [
    ("pose_L64", lambda: W.pose(40, 64, seed=3), 20),
    ("sparse_large_matchings", lambda: W.potts_er(700, 16, 0.08, seed=11), 6),
    ("pose_full_size", lambda: W.pose(200, 64, seed=0), 200)], ids=[c[0] for c in CASES[1:]] +
    ["pose_L64", "sparse_large_matchings", "pose_full_size"])
@pytest.mark.parametrize("rule", ["M", "U"])
def test_rule_on_the_mailbox_engine_is_bitwise_the_per_matching_engine(name, make, iters, rule):
    """FP32 iterate under (M) or (U) runs the persistent mailbox engine (two
    passes per update, or one and a reduction); its state, certified dual
    and rounding are bitwise those of the per-matching engine, whose traces
    the oracle pins."""
    _announce("rule mailbox", rule, name)
    model = make()
    out = []
    for engine in (M.ENGINE_PERSISTENT, M.ENGINE_STEP):
        with M.Solver.from_model(model) as s:
            s.set_option(M.OPT_RULE, M.RULE_M if rule == "M" else M.RULE_U)
            s.set_option(M.OPT_ENGINE, engine)
            s.iterate(iters)
            out.append((s.get_state(comp=True), s.dual_bound(), s.decode()))
    (a, da, deca), (b, db, decb) = out
    for x, y in zip(a, b):
        assert np.array_equal(x.view(np.uint32), y.view(np.uint32))
    assert da == db and np.array_equal(deca[0], decb[0])


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_one_iteration_dominance(seed):
    """From the same start, one iteration of (H) gives a dual at least that
    of (M), which is at least that of (U)."""
    _announce("dominance", seed)
    rng = np.random.default_rng(seed)
    model = _f64(W.uniform(int(rng.integers(5, 30)), int(rng.integers(2, 20)), seed=seed))
    d = {}
    for rule in (M.RULE_H, M.RULE_M, M.RULE_U):
        with M.Solver.from_model(model) as s:
            s.set_option(M.OPT_RULE, rule)
            s.iterate(1)
            d[rule] = s.dual_bound()
    assert d[M.RULE_H] >= d[M.RULE_M] - 1e-12 * abs(d[M.RULE_M])
    assert d[M.RULE_M] >= d[M.RULE_U] - 1e-12 * abs(d[M.RULE_U])


def test_rule_option_errors():
    _announce("rule errors")
    with M.Solver.from_model(W.uniform(6, 4, seed=1)) as s:
        with pytest.raises(M.MplpError) as ei:
            s.set_option(M.OPT_RULE, 3)
        assert ei.value.code == M.EINVAL
        s.set_option(M.OPT_RULE, M.RULE_M)
        with pytest.raises(M.MplpError) as ei:
            s.adjoint_forward(2, 1)
        assert ei.value.code == M.EINVAL
        s.set_option(M.OPT_RULE, M.RULE_H)
        s.adjoint_forward(2, 1)


@pytest.mark.parametrize("rule", ["M", "U"])
def test_rule_full_size_pose_matches_stored_oracle_trace(rule):
    """The pose workload at full size (n = 200, L = 64, 200 iterations from
    phi = 0) under (M) and (U): every iteration's dual within 1e-5 of the
    oracle's stored trace (tests/golden/make_golden.py, oracle only)."""
    import json
    import os
    _announce("full size rule", rule)
    g = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "pose_k200_l64_rules.json")))
    assert g["workload"] == "pose n=200 L=64 seed=0"
    ref = np.asarray(g["traces"][rule])
    model = W.pose(200, 64, seed=0)
    with M.Solver.from_model(model) as s:
        s.set_option(M.OPT_RULE, M.RULE_M if rule == "M" else M.RULE_U)
        tr = s.iterate_trace(200)
    rel = np.abs(tr - ref) / np.maximum(1.0, np.abs(ref))
    assert rel.max() <= 1e-5, (rel.max(), int(rel.argmax()))
