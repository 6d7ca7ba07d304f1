"""GPU tests of the structured Potts passes of the wave engine (Sec. 4: with
pairwise terms w [s != t] the message-passing minimization takes O(L)).

A batch built from one weight per edge (``mplpxx_batch_create_potts``) must
end bitwise equal to the dense batch on the expanded tables w [s != t], in
LDS mode and as teams through the mailboxes, on ties, negative and zero
weights, L = 1 and ragged L; its dual bounds must match the FP64 oracle on
the dense model to 1e-5.  The workgroup engine and L > 64 are refused."""
import numpy as np
import pytest

import oracle
from paper_2004_08227_amd import workloads as W

pytestmark = pytest.mark.gpu
M = pytest.importorskip("paper_2004_08227_amd")


def _announce(*a):
    print("CASE", *a, flush=True)


def _pairs(seed=0):
    """(weights model, dense model) pairs over the label counts the wave
    engine's lanes have to cover: 1, 2, ragged, and both sides of the
    row boundaries 16 and 32 of the second-minimum butterfly, up to 64."""
    out = []
    for k, (n, L, dens) in enumerate([(2, 1, 1.0), (5, 2, 1.0), (9, 7, 0.6), (12, 16, 1.0), (8, 17, 1.0),
                                       (10, 32, 0.8), (30, 33, 0.3), (16, 64, 1.0), (40, 13, 0.2), (3, 64, 1.0)]):
        out.append(W.potts_pure(n, L, dens, seed=seed + k))
    return out


def _run(models, potts, iters, opts):
    with M.Batch(models, potts=potts) as b:
        for k, v in opts.items():
            b.set_option(k, v)
        b.iterate(iters)
        info = dict(engine=b.info("engine"), lds_tasks=b.info("lds_tasks"), max_team=b.info("max_team"))
        states = [b.get_state(i, comp=True) for i in range(len(models))]
        duals = b.dual_bounds()
    return states, duals, info


MODES = {"lds": dict(engine=2, one_per_model=1),
         "team": dict(engine=2, lds=0, wave_lat_mb_us=1000.0),   # latency-bound plan: the largest teams
         "auto": dict()}


@pytest.mark.parametrize("mode", list(MODES))
def test_potts_batch_is_bitwise_the_dense_batch(mode):
    _announce("potts vs dense", mode)
    pairs = _pairs()
    weights = [p[0] for p in pairs]
    dense = [p[1] for p in pairs]
    iters = 6
    sp, dp, ip = _run(weights, True, iters, MODES[mode])
    sd, dd, idn = _run(dense, False, iters, MODES[mode])
    assert ip["engine"] == 2 and idn["engine"] == 2
    if mode == "lds":
        assert ip["lds_tasks"] == len(pairs)
    if mode == "team":
        assert ip["max_team"] > 1
    for i in range(len(pairs)):
        for a, b in zip(sp[i], sd[i]):
            assert np.array_equal(a.view(np.uint32), b.view(np.uint32)), (i, dense[i].name)
    assert np.array_equal(dp, dd)
    for i, mo in enumerate(dense):
        st, ref = oracle.run_model(mo, iters)
        assert abs(dp[i] - ref[-1]) <= 1e-5 * max(1.0, abs(ref[-1])), (i, dp[i], ref[-1])


def test_potts_ties_negative_and_zero_weights():
    """Integer unaries (many labels tie for the minimum, so the second
    minimum equals the first), negative weights, +0 and -0 weights."""
    _announce("potts ties / signs")
    rng = np.random.default_rng(5)
    pairs = []
    for k, (n, L) in enumerate([(10, 8), (14, 64), (6, 33)]):
        w_model, _ = W.potts_pure(n, L, 1.0, seed=50 + k, w_range=(-0.5, 1.0))
        un = rng.integers(0, 3, size=(n, L)).astype(np.float32)
        w = w_model.pairwise.copy()
        w[::5] = 0.0
        w[1::7] = -0.0
        w[2::9] = np.round(w[2::9])         # integer weights: ties through the passes too
        eye = np.eye(L, dtype=bool)[None]
        pw = np.where(eye, np.float32(0.0), w[:, None, None]).astype(np.float32)
        pairs.append((W.Model(n, L, w_model.edges, un, w, "ties_w"), W.Model(n, L, w_model.edges, un, pw, "ties")))
    iters = 8
    for mode in ("lds", "team"):
        sp, dp, _ = _run([p[0] for p in pairs], True, iters, MODES[mode])
        sd, dd, _ = _run([p[1] for p in pairs], False, iters, MODES[mode])
        for i in range(len(pairs)):
            for a, b in zip(sp[i], sd[i]):
                assert np.array_equal(a.view(np.uint32), b.view(np.uint32)), (mode, i)
        assert np.array_equal(dp, dd)
    for i, (_, mo) in enumerate(pairs):
        st, ref = oracle.run_model(mo, iters)
        assert abs(dp[i] - ref[-1]) <= 1e-5 * max(1.0, abs(ref[-1])), (i, dp[i], ref[-1])


def test_potts_full_size_complete_graph():
    """A complete Potts model at the pose size (200 nodes, 64 labels, 19900
    edges) with a mix of smaller ones: bitwise the dense batch, and the
    dual after 3 iterations within 1e-5 of the oracle on the dense model."""
    _announce("potts full size")
    pairs = [W.potts_pure(200, 64, 1.0, seed=11), W.potts_pure(120, 40, 0.5, seed=12),
             W.potts_pure(60, 21, 1.0, seed=13)]
    iters = 3
    sp, dp, _ = _run([p[0] for p in pairs], True, iters, {})
    sd, dd, _ = _run([p[1] for p in pairs], False, iters, {})
    for i in range(len(pairs)):
        for a, b in zip(sp[i], sd[i]):
            assert np.array_equal(a.view(np.uint32), b.view(np.uint32)), i
    assert np.array_equal(dp, dd)
    st, ref = oracle.run_model(pairs[0][1], iters)
    assert abs(dp[0] - ref[-1]) <= 1e-5 * max(1.0, abs(ref[-1])), (dp[0], ref[-1])


def test_potts_engine_and_size_errors():
    _announce("potts errors")
    w, _ = W.potts_pure(6, 8, 1.0, seed=1)
    with M.Batch([w], potts=True) as b:
        b.set_option("engine", 1)
        with pytest.raises(M.MplpError) as ei:
            b.iterate(1)
        assert ei.value.code == M.EINVAL
        b.set_option("engine", 0)
        b.iterate(1)
        assert b.info("engine") == 2
        assert b.info("table_bytes") == 4 * w.m
    big, _ = W.potts_pure(4, 65, 1.0, seed=2)
    with pytest.raises(M.MplpError) as ei:
        M.Batch([big], potts=True)
    assert ei.value.code == M.EINVAL
    with pytest.raises(ValueError):
        M.Batch([W.pose(4, 8, seed=1)], potts=True)


def test_potts_zero_messages_are_positive_zero():
    """All-zero unaries: every pass yields exactly 0 and every message is
    +0, as on the dense table (whose diagonal term is +0): the structured
    pass must not turn fl(0 - q) into -q, which is -0 for q = +0."""
    _announce("potts signed zeros")
    n, L = 5, 6
    w_model, d_model = W.potts_pure(n, L, 1.0, seed=3)
    z = np.zeros((n, L), np.float32)
    pair = (W.Model(n, L, w_model.edges, z, w_model.pairwise, "zero_w"),
            W.Model(n, L, d_model.edges, z, d_model.pairwise, "zero"))
    for mode in ("lds", "team"):
        sp, dp, _ = _run([pair[0]], True, 3, MODES[mode])
        sd, dd, _ = _run([pair[1]], False, 3, MODES[mode])
        assert not np.signbit(sd[0][1]).any() and not np.any(sd[0][1])
        for a, b in zip(sp[0], sd[0]):
            assert np.array_equal(a.view(np.uint32), b.view(np.uint32)), mode


@pytest.mark.parametrize("mode", ["lds", "team"])
def test_potts_reset_and_timeout(mode):
    """A spin limit of 1 (set from the host) makes the waits of the Potts
    kernel give up: the launch reports MPLPXX_ETIMEOUT and every wave exits;
    after a reset the batch reproduces its first run bit for bit."""
    _announce("potts reset/timeout", mode)
    weights = [p[0] for p in _pairs(seed=3)]
    with M.Batch(weights, potts=True) as b:
        for k, v in MODES[mode].items():
            b.set_option(k, v)
        b.iterate(3)
        d3 = b.dual_bounds()
        b.reset()
        b.set_option("spin_limit", 1)
        with pytest.raises(M.MplpError) as ei:
            b.iterate(3)
        assert ei.value.code == M.ETIMEOUT
        b.set_option("spin_limit", 0)
        b.reset()
        b.iterate(3)
        assert np.array_equal(b.dual_bounds(), d3)


# ---------------------------------------------------------------------------
# Single-model Potts handles (mplpxx_create_potts) on the mailbox engine
# ---------------------------------------------------------------------------
def _solver_run(make, iters):
    with make() as s:
        s.iterate(iters)
        U, phi, c = s.get_state(comp=True)
        d = s.dual_bound()
        lab, e = s.decode()
        info = (s.info("engine"), s.info("grid"), s.info("threads"))
    return (U, phi, c), d, (lab, e), info


SOLVER_CASES = [(2, 1, 1.0), (5, 2, 1.0), (9, 7, 0.6), (12, 16, 1.0), (8, 17, 1.0), (10, 32, 0.8), (30, 33, 0.3),
                (16, 64, 1.0), (200, 64, 1.0), (120, 40, 0.5),
                (600, 8, 1.0)]   # 300 edges per matching: more workgroups than CUs, messages in HBM


@pytest.mark.parametrize("n,L,p", SOLVER_CASES, ids=[f"n{n}_L{L}_p{p}" for n, L, p in SOLVER_CASES])
def test_potts_solver_is_bitwise_the_dense_solver(n, L, p):
    _announce("potts solver", n, L, p)
    w, d = W.potts_pure(n, L, p, seed=n + L)
    iters = 4 if n >= 200 else 7
    sp, dp, lp, ip = _solver_run(lambda: M.Solver.from_potts(w), iters)
    sd, dd, ld, idn = _solver_run(lambda: M.Solver.from_model(d), iters)
    # default engine: tiles formed from the weights up to 32 labels (on four
    # compute waves, or on one at up to 16 labels when a matching has more
    # edges than there are compute units), one wave in label order above
    import torch
    step_ptr, _ = oracle.schedule(n, np.asarray(d.edges), "greedy")
    one_wave = L <= 16 and int(np.diff(step_ptr).max()) > torch.cuda.get_device_properties(0).multi_processor_count
    assert ip[0] == M.ENGINE_PERSISTENT and ip[2] == (256 if L <= 32 and not one_wave else 64)
    for a, b in zip(sp, sd):
        assert np.array_equal(a.view(np.uint32), b.view(np.uint32))
    assert dp == dd
    assert np.array_equal(lp[0], ld[0]) and lp[1] == ld[1]
    # the other single-model Potts engine
    def other():
        s = M.Solver.from_potts(w)
        s.set_option(M.OPT_THREADS, 64 if L <= 32 else 256)
        return s
    so, do, lo, io = _solver_run(other, iters)
    assert io[2] == (64 if L <= 32 else 256)
    for a, b in zip(so, sd):
        assert np.array_equal(a.view(np.uint32), b.view(np.uint32))
    assert do == dd
    # the same model as a Potts batch: bitwise the same state
    with M.Batch([w], potts=True) as bt:
        bt.iterate(iters)
        sb = bt.get_state(0, comp=True)
    for a, b in zip(sp, sb):
        assert np.array_equal(a.view(np.uint32), b.view(np.uint32))
    if n <= 200:
        st, ref = oracle.run_model(d, iters)
        assert abs(dp - ref[-1]) <= 1e-5 * max(1.0, abs(ref[-1])), (dp, ref[-1])


def test_potts_solver_gap_state_and_timeout():
    _announce("potts solver gap/state/timeout")
    w, d = W.potts_pure(40, 12, 0.5, seed=4)
    with M.Solver.from_potts(w) as s, M.Solver.from_model(d) as t:
        gp = s.iterate_gap(5)
        gd = t.iterate_gap(5)
        for a, b in zip(gp, gd):
            assert np.array_equal(np.asarray(a), np.asarray(b))
        U, phi, c = s.get_state(comp=True)
        s.iterate(3)
        ref = s.get_state(comp=True)
        s.set_state(U, phi, c)
        s.set_option(M.OPT_SPIN_LIMIT, 1)
        with pytest.raises(M.MplpError) as ei:
            s.iterate(3)
        assert ei.value.code == M.ETIMEOUT
        s.set_option(M.OPT_SPIN_LIMIT, 0)
        s.set_state(U, phi, c)
        s.iterate(3)
        for a, b in zip(s.get_state(comp=True), ref):
            assert np.array_equal(a.view(np.uint32), b.view(np.uint32))


def test_potts_solver_rejects_dense_only_calls():
    _announce("potts solver errors")
    w, _ = W.potts_pure(8, 6, 1.0, seed=5)
    with M.Solver.from_potts(w) as s:
        for key, val in ((M.OPT_ENGINE, M.ENGINE_STEP), (M.OPT_THREADS, 512), (M.OPT_RULE, M.RULE_M)):
            with pytest.raises(M.MplpError) as ei:
                s.set_option(key, val)
            assert ei.value.code == M.EINVAL
        with pytest.raises(M.MplpError) as ei:
            s.iterate_trace(2)
        assert ei.value.code == M.EINVAL
        with pytest.raises(M.MplpError) as ei:
            s.adjoint_forward(2, 1)
        assert ei.value.code == M.EINVAL
        s.iterate(1)


@pytest.mark.parametrize("L", [1, 2, 5, 16, 17, 33, 64])
def test_potts_single_edge_update_reaches_the_map(L):
    """One (H) update of a single edge is block-optimal (Sec. 4): the dual
    equals min_{s,t} theta_u(s) + theta_v(t) + w [s != t], brute force, for
    positive, negative and zero weights (FP32 tolerance)."""
    _announce("potts single edge", L)
    rng = np.random.default_rng(L)
    for w in (0.7, -0.3, 0.0, float(rng.uniform(0.1, 2.0))):
        un = rng.random((2, L)).astype(np.float32)
        model = W.Model(2, L, np.array([[0, 1]], np.int32), un, np.array([w], np.float32), "edge")
        with M.Solver.from_potts(model) as s:
            s.iterate(1)
            d = s.dual_bound()
        th = np.where(np.eye(L, dtype=bool), 0.0, np.float64(np.float32(w)))
        g = un[0].astype(np.float64)[:, None] + un[1].astype(np.float64)[None, :] + th
        assert abs(d - g.min()) <= 1e-5 * max(1.0, abs(g.min())), (L, w, d, g.min())


def test_potts_edgeless_models():
    """No edges (single handle and inside a batch) and a single node: the
    dual bound is the sum of the unary minima, before and after iterating."""
    _announce("potts edgeless")
    rng = np.random.default_rng(9)
    for n, L in ((1, 5), (4, 64), (7, 3)):
        un = rng.random((n, L)).astype(np.float32)
        model = W.Model(n, L, np.zeros((0, 2), np.int32), un, np.zeros(0, np.float32), "edgeless")
        want = float(np.sum(un.astype(np.float64).min(axis=1)))
        with M.Solver.from_potts(model) as s:
            assert s.dual_bound() == pytest.approx(want, rel=1e-12)
            s.iterate(3)
            assert s.dual_bound() == pytest.approx(want, rel=1e-12)
            lab, e = s.decode()
            assert np.array_equal(lab, un.argmin(axis=1))
        w, _ = W.potts_pure(9, L, 1.0, seed=n)
        with M.Batch([model, w], potts=True) as b:
            b.iterate(3)
            d = b.dual_bounds()
        assert d[0] == pytest.approx(want, rel=1e-12)
