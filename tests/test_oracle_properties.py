"""Property tests of the FP64 oracle on randomly drawn tiny models (hypothesis).

The seeded pins of test_oracle_pins.py check each statement of the paper on a
few fixed models; here hypothesis searches (and shrinks) over graph shape,
edge orientation, label count and cost distribution for a counterexample to
the same statements:

* the dual bound of Eq. (3) never decreases, neither over iterations nor over
  single updates (Sec. 5), for each of the updates (H), (M), (U) of Sec. 4;
* it stays below the energy of every labelling, in particular of the MAP
  labelling found by brute force and of the rounding of Eq. (5);
* reparametrization leaves every labelling's energy unchanged (Eq. 2);
* one iteration of (H) from any state dominates one of (M), which dominates
  (U) (Thm. 2);
* the schedule of Alg. 1 is a sequence of matchings covering every edge once,
  for the greedy and the colouring rule.
"""
import numpy as np
import pytest

hyp = pytest.importorskip("hypothesis")
from hypothesis import HealthCheck, given, settings  # noqa: E402
from hypothesis import strategies as st  # noqa: E402

import oracle  # noqa: E402
from paper_2004_08227_amd import workloads as W  # noqa: E402

SETTINGS = settings(max_examples=150, deadline=None, database=None,
                    suppress_health_check=[HealthCheck.too_slow])


@st.composite
def tiny_models(draw, max_n=5, max_L=3):
    """A model with 2..max_n nodes, 1..max_L labels, a random edge subset
    given in random orientation, and costs of one of three kinds: integers
    in [-3, 3] (many ties), dyadic numbers in [-2, 2], or uniform floats."""
    n = draw(st.integers(2, max_n))
    L = draw(st.integers(1, max_L))
    pairs = [(u, v) for u in range(n) for v in range(u + 1, n)]
    keep = draw(st.lists(st.booleans(), min_size=len(pairs), max_size=len(pairs)))
    flips = draw(st.lists(st.booleans(), min_size=len(pairs), max_size=len(pairs)))
    edges = [(v, u) if f else (u, v) for (u, v), k, f in zip(pairs, keep, flips) if k]
    kind = draw(st.sampled_from(["integer", "dyadic", "uniform"]))
    rng = np.random.default_rng(draw(st.integers(0, 2**32 - 1)))
    m = len(edges)
    if kind == "integer":
        un = rng.integers(-3, 4, size=(n, L)).astype(np.float64)
        pw = rng.integers(-3, 4, size=(m, L, L)).astype(np.float64)
    elif kind == "dyadic":
        un = rng.integers(-16, 17, size=(n, L)) / 8.0
        pw = rng.integers(-16, 17, size=(m, L, L)) / 8.0
    else:
        un = rng.random((n, L))
        pw = rng.random((m, L, L))
    e = np.asarray(edges, dtype=np.int32).reshape(m, 2)
    return W.Model(n, L, e, un, pw.reshape(m, L, L), f"hyp_{kind}")


def _tol(model):
    scale = 1.0 + np.abs(model.unaries).sum() + np.abs(model.pairwise).sum()
    return 1e-12 * scale


@SETTINGS
@given(tiny_models(), st.sampled_from("HMU"))
def test_dual_rises_and_stays_below_every_energy(model, rule):
    st_, tr = oracle.run_model(model, 6, rule=rule)
    tol = _tol(model)
    d0 = oracle.State(model).dual()
    assert tr[0] >= d0 - tol
    assert np.all(np.diff(tr) >= -tol)
    e_map, _ = oracle.bruteforce(model)
    assert tr[-1] <= e_map + tol
    labels = st_.decode()
    assert st_.energy(labels) >= e_map - tol
    # reparametrization keeps every labelling's energy (Eq. 2)
    rng = np.random.default_rng(model.n * 7 + model.L)
    for _ in range(4):
        y = rng.integers(0, model.L, size=model.n).astype(np.int32)
        assert abs(st_.energy(y, reparametrized=True) - st_.energy(y)) <= tol


@SETTINGS
@given(tiny_models(), st.sampled_from("HMU"))
def test_every_single_update_keeps_the_dual_from_falling(model, rule):
    s = oracle.State(model)
    tol = _tol(model)
    d = s.dual()
    # edges one at a time in schedule order, each a block-coordinate step
    for i in s.order:
        u, v = s.edges[i]
        Te, hu, hv = oracle.update(rule, s.Te[i], s.Tu[u], s.Tu[v])
        s.Te[i], s.Tu[u], s.Tu[v] = Te, hu, hv
        d_new = s.dual()
        assert d_new >= d - tol
        d = d_new


@SETTINGS
@given(tiny_models(), st.integers(0, 3))
def test_one_handshake_iteration_dominates_mplp_and_uniform(model, warm):
    base = oracle.State(model)
    base.run(warm, rule="M")
    ds = {}
    for rule in "HMU":
        s = oracle.State(model)
        s.Tu[:] = base.Tu
        s.Te[:] = base.Te
        s.run(1, rule=rule)
        ds[rule] = s.dual()
    tol = _tol(model)
    assert ds["H"] >= ds["M"] - tol and ds["M"] >= ds["U"] - tol


@SETTINGS
@given(st.integers(2, 12), st.floats(0.0, 1.0), st.integers(0, 2**32 - 1), st.sampled_from(["greedy", "color"]))
def test_schedule_is_a_sequence_of_matchings_covering_every_edge_once(n, p, seed, kind):
    rng = np.random.default_rng(seed)
    iu, iv = np.triu_indices(n, 1)
    keep = rng.random(iu.shape[0]) < p
    edges = np.stack([iu[keep], iv[keep]], axis=1).astype(np.int32)
    step_ptr, order = oracle.schedule(n, edges, kind)
    assert step_ptr[0] == 0 and step_ptr[-1] == edges.shape[0]
    assert np.array_equal(np.sort(order), np.arange(edges.shape[0]))
    for k in range(step_ptr.shape[0] - 1):
        nodes = edges[order[step_ptr[k]:step_ptr[k + 1]]].ravel()
        assert step_ptr[k + 1] > step_ptr[k]
        assert np.unique(nodes).size == nodes.size
