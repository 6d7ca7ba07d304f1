"""GPU tests of truncated linear pairwise costs w min(|s - t|, tau) (Sec. 4:
absolute-difference costs are among those whose message passing takes O(L)).

The structured passes in label order (a min-plus distance transform per
pass, O(L) work and O(log L) steps) form their sums in another order than
the dense passes, so their reference is the FP64 oracle on the expanded FP32
tables, at the FP32 parity bar: the certified dual and every reparametrized
unary and pairwise cost within 1e-5 (relative to max(1, |value|)), on the
single-model engine and on the batched wave engine (models in LDS and split
over teams), with ragged label counts, ties, zero weights, truncation at 0,
below 1 (a Potts cost) and beyond the label range (plain absolute
difference).  The single-model engine with tiles formed from (w, tau) (the
default) gives the dense engine's bits on the expanded tables, and the
oracle's bar as well."""
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
    ("complete_L13_tau3.5", lambda: W.trunc_linear(40, 13, 1.0, seed=1, tau=3.5), 20),
    ("er30_L33_tau5", lambda: W.trunc_linear(60, 33, 0.3, seed=2, tau=5.0), 15),
    ("complete_L64_absdiff", lambda: W.trunc_linear(24, 64, 1.0, seed=3, tau=100.0), 10),
    ("complete_L16_tau0", lambda: W.trunc_linear(30, 16, 1.0, seed=4, tau=0.0), 5),
    ("complete_L20_tau0.5", lambda: W.trunc_linear(30, 20, 1.0, seed=5, tau=0.5), 10),
    ("integer_ties_L10", lambda: W.trunc_linear(20, 10, 1.0, seed=6, tau=3.0, integer=True), 15),
    ("er50_L48_tau6", lambda: W.trunc_linear(36, 48, 0.5, seed=7, tau=6.0), 10),
    ("single_label", lambda: W.trunc_linear(8, 1, 1.0, seed=8, tau=2.0), 3),
]


def _check_state(dense, iters, d, U, phi, Uc):
    st, ref = oracle.run_model(dense, iters)
    assert abs(d - ref[-1]) <= 1e-5 * max(1.0, abs(ref[-1])), (d, ref[-1])
    eu = SP.worst(SP.gpu_unaries(U, Uc), st.Tu)
    ep = SP.worst(SP.gpu_pairwise(dense.pairwise, phi), st.Te)
    return eu, ep


@pytest.mark.parametrize("threads", [64, 256], ids=["label_order", "formed_tiles"])
@pytest.mark.parametrize("name,make,iters", CASES, ids=[c[0] for c in CASES])
def test_single_model_engine_matches_oracle_on_expanded_tables(name, make, iters, threads):
    _announce("trunc linear single", name, "threads", threads)
    params, dense = make()
    with M.Solver.from_structured(params, M.COST_TRUNC_LINEAR) as s:
        s.set_option(M.OPT_THREADS, threads)
        assert s.info("threads") == threads
        s.iterate(iters)
        d = s.dual_bound()
        U, phi, Uc = s.get_state(comp=True)
        labels, energy = s.decode()
    eu, ep = _check_state(dense, iters, d, U, phi, Uc)
    print(f"{name} threads {threads}: unaries {eu:.2e}, pairwise {ep:.2e}", flush=True)
    assert eu <= SP.TOL and ep <= SP.TOL
    # the rounding's energy is Eq. (1) on the expanded costs
    assert abs(energy - oracle.energy(dense, labels)) <= 1e-5 * max(1.0, abs(energy))
    if threads == 256:
        # formed tiles: the dense engine's bits on the expanded tables
        with M.Solver.from_model(dense) as sd:
            sd.iterate(iters)
            assert sd.dual_bound() == d
            for a, b in zip(sd.get_state(comp=True), (U, phi, Uc)):
                assert np.array_equal(a.view(np.uint32), b.view(np.uint32))
            assert np.array_equal(sd.decode()[0], labels)


def test_formed_tiles_are_the_default():
    params, _ = W.trunc_linear(12, 9, 1.0, seed=40, tau=2.0)
    with M.Solver.from_structured(params, M.COST_TRUNC_LINEAR) as s:
        assert s.info("threads") == 256


STRUCT_16 = [
    ("potts", M.COST_POTTS, lambda: W.potts_pure(700, 16, 0.1, seed=41)),
    ("trunc_linear", M.COST_TRUNC_LINEAR, lambda: W.trunc_linear(700, 16, 0.1, seed=42, tau=5.0)),
    ("trunc_quad", M.COST_TRUNC_QUAD, lambda: W.trunc_quad(700, 16, 0.1, seed=43, tau=20.0)),
]


@pytest.mark.parametrize("name,kind,make", STRUCT_16, ids=[c[0] for c in STRUCT_16])
def test_formed_tiles_one_compute_wave_at_16_labels(name, kind, make):
    # 16 labels and matchings with more edges than there are compute units:
    # the formed tiles run one compute wave by default, like the tables, and
    # give the dense handle's bits
    _announce("formed tiles one wave", name)
    params, dense = make()
    iters = 6
    with M.Solver.from_structured(params, kind) as s, M.Solver.from_model(dense) as sd:
        # (the default takes one wave only when a matching outnumbers the CUs)
        assert s.info("threads") == 64 and sd.info("threads") == 64
        s.iterate(iters)
        sd.iterate(iters)
        assert s.dual_bound() == sd.dual_bound()
        for a, b in zip(sd.get_state(comp=True), s.get_state(comp=True)):
            assert np.array_equal(a.view(np.uint32), b.view(np.uint32))
        # four compute waves (threads 256) give the same bits
        s.set_option(M.OPT_THREADS, 256)
        assert s.info("threads") == 256
        U0 = dense.unaries.copy()
        s.set_state(U0, np.zeros((dense.m, 2, dense.L), np.float32))
        s.iterate(iters)
        for a, b in zip(sd.get_state(comp=True), s.get_state(comp=True)):
            assert np.array_equal(a.view(np.uint32), b.view(np.uint32))


def test_per_edge_truncation_and_zero_weights():
    _announce("trunc linear per-edge tau")
    rng = np.random.default_rng(11)
    params, _ = W.trunc_linear(32, 24, 1.0, seed=11, tau=1.0)
    prm = params.pairwise.copy()
    prm[:, 1] = rng.choice([0.0, 0.75, 2.0, 5.5, 30.0], size=prm.shape[0]).astype(np.float32)
    prm[::7, 0] = 0.0
    params = W.Model(params.n, params.L, params.edges, params.unaries, prm)
    d_ = np.abs(np.arange(24)[:, None] - np.arange(24)[None, :]).astype(np.float32)
    dense = W.Model(params.n, params.L, params.edges, params.unaries,
                    (prm[:, 0, None, None] * np.minimum(d_[None], prm[:, 1, None, None])).astype(np.float32))
    with M.Solver.from_structured(params, M.COST_TRUNC_LINEAR) as s:
        s.iterate(12)
        d = s.dual_bound()
        U, phi, Uc = s.get_state(comp=True)
    eu, ep = _check_state(dense, 12, d, U, phi, Uc)
    assert eu <= SP.TOL and ep <= SP.TOL


def test_zero_truncation_gives_the_unary_bound():
    """tau = 0 makes every pairwise cost 0: D_K = sum_u min theta_u."""
    _announce("trunc linear tau=0 bound")
    params, dense = W.trunc_linear(20, 12, 1.0, seed=12, tau=0.0)
    with M.Solver.from_structured(params, M.COST_TRUNC_LINEAR) as s:
        s.iterate(4)
        d = s.dual_bound()
    assert abs(d - float(params.unaries.astype(np.float64).min(axis=1).sum())) <= 1e-5


MODES = {"lds": dict(engine=2, one_per_model=1),
         "team": dict(engine=2, lds=0, wave_lat_mb_us=1000.0),   # latency-bound plan: the largest teams
         "auto": dict()}


@pytest.mark.parametrize("mode", list(MODES))
def test_batched_wave_engine_matches_oracle(mode):
    """A batch of truncated linear models of mixed sizes, with every model in
    LDS, with teams through the mailboxes, and as planned."""
    _announce("trunc linear batch", mode)
    pairs = [W.trunc_linear(12, 5, 1.0, seed=20, tau=2.0), W.trunc_linear(30, 33, 0.5, seed=21, tau=4.0),
             W.trunc_linear(25, 64, 1.0, seed=22, tau=100.0), W.trunc_linear(60, 64, 1.0, seed=23, tau=8.0),
             W.trunc_linear(16, 17, 1.0, seed=24, tau=0.5, integer=True)]
    params = [p for p, _ in pairs]
    iters = 8
    with M.Batch(params, kind=M.COST_TRUNC_LINEAR) as b:
        for k, v in MODES[mode].items():
            b.set_option(k, v)
        b.iterate(iters)
        if mode == "lds":
            assert b.info("lds_tasks") == len(pairs)
        if mode == "team":
            assert b.info("max_team") > 1
        duals = b.dual_bounds()
        states = [b.get_state(i, comp=True) for i in range(len(params))]
    for i, (_, dense) in enumerate(pairs):
        U, phi, Uc = states[i]
        eu, ep = _check_state(dense, iters, duals[i], U, phi, Uc)
        print(f"batch model {i} (n={dense.n}, L={dense.L}): unaries {eu:.2e}, pairwise {ep:.2e}", flush=True)
        assert eu <= SP.TOL and ep <= SP.TOL


def test_batched_and_single_model_engines_agree_bitwise():
    """The two engines in label order run the same passes in the same order
    per label."""
    _announce("trunc linear batch vs single")
    params, _ = W.trunc_linear(40, 29, 0.6, seed=30, tau=3.0)
    with M.Solver.from_structured(params, M.COST_TRUNC_LINEAR) as s:
        s.set_option(M.OPT_THREADS, 64)
        s.iterate(6)
        Ua, pa = s.get_state()
    with M.Batch([params], kind=M.COST_TRUNC_LINEAR) as b:
        b.iterate(6)
        Ub, pb = b.get_state(0)
    assert np.array_equal(Ua, Ub) and np.array_equal(pa, pb)
