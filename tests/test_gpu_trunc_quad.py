"""GPU tests of truncated quadratic pairwise costs w min((s - t)^2, tau) (Sec.
4: quadratic costs are among those whose message passing needs no L x L
table).

The structured passes form every candidate fl(x(t) + fl(w min((s - t)^2,
tau))) from the two parameters of the edge, with the same single IEEE add as
the dense passes, so the reference is twofold: the dense engine on the
expanded FP32 tables, bitwise (state, certified dual, rounding), and the FP64
oracle on the same tables at the FP32 parity bar (the certified dual and
every reparametrized unary and pairwise cost within 1e-5 relative to max(1,
|value|)).  Covered: the single-model engine and the batched wave engine
(models in LDS, split over teams, as planned), ragged label counts, integer
ties, zero weights, truncation at 0, below 1 (a Potts cost), per-edge tau and
tau beyond (L - 1)^2 (the plain quadratic cost)."""
import numpy as np
import pytest

import oracle
from paper_2004_08227_amd import workloads as W
from tests import state_parity as SP

pytestmark = pytest.mark.gpu
M = pytest.importorskip("paper_2004_08227_amd")


def _announce(*a):
    print("CASE", *a, flush=True)


CASES = [
    ("complete_L13_tau9", lambda: W.trunc_quad(40, 13, 1.0, seed=1, tau=9.0), 20),
    ("er30_L33_tau30", lambda: W.trunc_quad(60, 33, 0.3, seed=2, tau=30.0), 15),
    ("complete_L64_quadratic", lambda: W.trunc_quad(24, 64, 1.0, seed=3, tau=5000.0), 10),
    ("complete_L16_tau0", lambda: W.trunc_quad(30, 16, 1.0, seed=4, tau=0.0), 5),
    ("complete_L20_tau0.5", lambda: W.trunc_quad(30, 20, 1.0, seed=5, tau=0.5), 10),
    ("integer_ties_L10", lambda: W.trunc_quad(20, 10, 1.0, seed=6, tau=9.0, integer=True), 15),
    ("er50_L48_tau100", lambda: W.trunc_quad(36, 48, 0.5, seed=7, tau=100.0), 10),
    ("single_label", lambda: W.trunc_quad(8, 1, 1.0, seed=8, tau=4.0), 3),
]


def _check_oracle(dense, iters, d, U, phi, Uc):
    st, ref = oracle.run_model(dense, iters)
    assert abs(d - ref[-1]) <= 1e-5 * max(1.0, abs(ref[-1])), (d, ref[-1])
    eu = SP.worst(SP.gpu_unaries(U, Uc), st.Tu)
    ep = SP.worst(SP.gpu_pairwise(dense.pairwise, phi), st.Te)
    return eu, ep


def _run_dense(dense, iters):
    with M.Solver.from_model(dense) as s:
        s.iterate(iters)
        return s.dual_bound(), s.get_state(comp=True), s.decode()


@pytest.mark.parametrize("name,make,iters", CASES, ids=[c[0] for c in CASES])
def test_single_model_engine_bitwise_dense_and_oracle(name, make, iters):
    _announce("trunc quad single", name)
    params, dense = make()
    with M.Solver.from_structured(params, M.COST_TRUNC_QUAD) as s:
        s.iterate(iters)
        d = s.dual_bound()
        U, phi, Uc = s.get_state(comp=True)
        labels, energy = s.decode()
    dd, (Ud, phid, Ucd), (labd, ed) = _run_dense(dense, iters)
    assert np.array_equal(U.view(np.uint32), Ud.view(np.uint32))
    assert np.array_equal(Uc.view(np.uint32), Ucd.view(np.uint32))
    assert np.array_equal(phi.view(np.uint32), phid.view(np.uint32))
    assert d == dd and np.array_equal(labels, labd) and energy == ed
    eu, ep = _check_oracle(dense, iters, d, U, phi, Uc)
    print(f"{name}: bitwise = dense engine; oracle: unaries {eu:.2e}, pairwise {ep:.2e}", flush=True)
    assert eu <= SP.TOL and ep <= SP.TOL
    assert abs(energy - oracle.energy(dense, labels)) <= 1e-5 * max(1.0, abs(energy))


def test_per_edge_truncation_and_zero_weights():
    _announce("trunc quad per-edge tau")
    rng = np.random.default_rng(11)
    params, _ = W.trunc_quad(32, 24, 1.0, seed=11, tau=1.0)
    prm = params.pairwise.copy()
    prm[:, 1] = rng.choice([0.0, 0.75, 2.0, 5.5, 30.0, 900.0], size=prm.shape[0]).astype(np.float32)
    prm[::7, 0] = 0.0
    params = W.Model(params.n, params.L, params.edges, params.unaries, prm)
    d_ = (np.arange(24)[:, None] - np.arange(24)[None, :]).astype(np.float32)
    dense = W.Model(params.n, params.L, params.edges, params.unaries,
                    (prm[:, 0, None, None] * np.minimum((d_ * d_)[None], prm[:, 1, None, None])).astype(np.float32))
    with M.Solver.from_structured(params, M.COST_TRUNC_QUAD) as s:
        s.iterate(12)
        d = s.dual_bound()
        U, phi, Uc = s.get_state(comp=True)
    dd, (Ud, phid, _), _ = _run_dense(dense, 12)
    assert d == dd and np.array_equal(U, Ud) and np.array_equal(phi, phid)
    eu, ep = _check_oracle(dense, 12, d, U, phi, Uc)
    assert eu <= SP.TOL and ep <= SP.TOL


def test_zero_truncation_gives_the_unary_bound():
    """tau = 0 makes every pairwise cost 0: D_K = sum_u min theta_u."""
    _announce("trunc quad tau=0 bound")
    params, _ = W.trunc_quad(20, 12, 1.0, seed=12, tau=0.0)
    with M.Solver.from_structured(params, M.COST_TRUNC_QUAD) as s:
        s.iterate(4)
        d = s.dual_bound()
    assert abs(d - float(params.unaries.astype(np.float64).min(axis=1).sum())) <= 1e-5


MODES = {"lds": dict(engine=2, one_per_model=1),
         "team": dict(engine=2, lds=0, wave_lat_mb_us=1000.0),   # latency-bound plan: the largest teams
         "auto": dict()}


@pytest.mark.parametrize("mode", list(MODES))
def test_batched_wave_engine_bitwise_dense_and_oracle(mode):
    """A batch of truncated quadratic models of mixed sizes, with every model
    in LDS, with teams through the mailboxes, and as planned: bitwise the
    dense batch on the expanded tables under the same options, and the
    oracle at the FP32 bar."""
    _announce("trunc quad batch", mode)
    pairs = [W.trunc_quad(12, 5, 1.0, seed=20, tau=4.0), W.trunc_quad(30, 33, 0.5, seed=21, tau=40.0),
             W.trunc_quad(25, 64, 1.0, seed=22, tau=5000.0), W.trunc_quad(60, 64, 1.0, seed=23, tau=64.0),
             W.trunc_quad(16, 17, 1.0, seed=24, tau=0.5, integer=True)]
    params = [p for p, _ in pairs]
    iters = 8
    with M.Batch(params, kind=M.COST_TRUNC_QUAD) as b:
        for k, v in MODES[mode].items():
            b.set_option(k, v)
        b.iterate(iters)
        if mode == "lds":
            assert b.info("lds_tasks") == len(pairs)
        if mode == "team":
            assert b.info("max_team") > 1
        duals = b.dual_bounds()
        states = [b.get_state(i, comp=True) for i in range(len(params))]
    with M.Batch([dn for _, dn in pairs]) as bd:
        for k, v in MODES[mode].items():
            bd.set_option(k, v)
        bd.iterate(iters)
        duals_d = bd.dual_bounds()
        states_d = [bd.get_state(i, comp=True) for i in range(len(params))]
    for i, (_, dense) in enumerate(pairs):
        U, phi, Uc = states[i]
        Ud, phid, Ucd = states_d[i]
        assert duals[i] == duals_d[i]
        assert np.array_equal(U, Ud) and np.array_equal(phi, phid) and np.array_equal(Uc, Ucd)
        eu, ep = _check_oracle(dense, iters, duals[i], U, phi, Uc)
        print(f"batch model {i} (n={dense.n}, L={dense.L}): unaries {eu:.2e}, pairwise {ep:.2e}", flush=True)
        assert eu <= SP.TOL and ep <= SP.TOL


def test_batched_and_single_model_engines_agree_bitwise():
    _announce("trunc quad batch vs single")
    params, _ = W.trunc_quad(40, 29, 0.6, seed=30, tau=20.0)
    with M.Solver.from_structured(params, M.COST_TRUNC_QUAD) as s:
        s.iterate(6)
        Ua, pa = s.get_state()
    with M.Batch([params], kind=M.COST_TRUNC_QUAD) as b:
        b.iterate(6)
        Ub, pb = b.get_state(0)
    assert np.array_equal(Ua, Ub) and np.array_equal(pa, pb)


@pytest.mark.parametrize("L,tau", [(7, 9.0), (16, 30.0), (33, 5000.0), (64, 64.0)])
def test_formed_tiles_and_label_order_engines_agree_bitwise(L, tau):
    """The single-model engine with four compute waves whose tiles are formed
    from (w, tau) (threads 256, the default) and the one-wave label-order
    engine (threads 64) give the same bits, and both the dense engine's."""
    _announce("trunc quad formed tiles", L, tau)
    params, dense = W.trunc_quad(30, L, 1.0, seed=50 + L, tau=tau)
    out = []
    for nt in (256, 64):
        with M.Solver.from_structured(params, M.COST_TRUNC_QUAD) as s:
            s.set_option(M.OPT_THREADS, nt)
            assert s.info("threads") == nt
            s.iterate(8)
            out.append((s.dual_bound(), s.get_state(comp=True)))
    dd, st_d, _ = _run_dense(dense, 8)
    for d, st in out:
        assert d == dd
        for a, b in zip(st, st_d):
            assert np.array_equal(a.view(np.uint32), b.view(np.uint32))
