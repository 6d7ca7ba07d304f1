"""GPU tests of the adjoint of K unrolled MPLP++ iterations.

D_K is piecewise linear in the costs, so inside a linear piece a central
finite difference of the FP64 oracle is exact up to rounding.  The FP64
adjoint must match such differences coordinate by coordinate on a small
model.  On the differentiation workload (n=100, L=32, K=50, checkpoints
every 10) the gradient of an FP32 handle (by default that of its exactly
widened FP64 twin run) must match stored FP64 differences along seeded
sparse directions and coordinates to 1e-4, and along dense directions to
1e-4 plus the rounding noise of the differences themselves; the gradient
of the FP32 run itself must stay within a few percent of it.  Checkpoint
spacing must not change a bit."""
import json
import os

import numpy as np
import pytest

import oracle
from paper_2004_08227_amd import workloads as W

pytestmark = pytest.mark.gpu
M = pytest.importorskip("paper_2004_08227_amd")
GOLD = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def _announce(*a):
    print("CASE", *a, flush=True)


def _grad(model, K, every, adjoint_f64=1):
    with M.Solver.from_model(model) as s:
        s.set_option(M.OPT_ADJOINT_F64, adjoint_f64)
        loss = s.adjoint_forward(K, every)
        gu, gp = s.adjoint_backward()
    return loss, gu, gp


def _fd(model, K, du, dp, h):
    base = model.astype(np.float64)
    plus = W.Model(base.n, base.L, base.edges, base.unaries + h * du, base.pairwise + h * dp)
    minus = W.Model(base.n, base.L, base.edges, base.unaries - h * du, base.pairwise - h * dp)
    return (oracle.dual_after(plus, K) - oracle.dual_after(minus, K)) / (2 * h)


def test_fp64_adjoint_matches_finite_differences_per_coordinate():
    _announce("fp64 adjoint all coordinates")
    model = W.uniform(9, 4, seed=21, dtype=np.float64)
    K, every = 6, 2
    loss, gu, gp = _grad(model, K, every)
    st, tr = oracle.run_model(model, K)
    assert abs(loss - st.dual()) <= 1e-12 * max(1, abs(loss))
    h = 1e-7
    bad = 0
    total = 0
    for arr, g in ((model.unaries, gu), (model.pairwise, gp)):
        for idx in np.ndindex(arr.shape):
            du = np.zeros(model.unaries.shape)
            dp = np.zeros(model.pairwise.shape)
            (du if arr is model.unaries else dp)[idx] = 1.0
            fd = _fd(model, K, du, dp, h)
            total += 1
            if abs(g[idx] - fd) > 1e-6 * max(1.0, abs(fd)):
                bad += 1
    # a step may cross a kink of the piecewise-linear D_K for a few coordinates
    assert bad <= max(1, total // 200), (bad, total)


def test_checkpoint_spacing_and_repeats_are_bitwise_identical():
    for dtype, f64 in ((np.float64, 1), (np.float32, 1), (np.float32, 0)):
        model = W.uniform(14, 6, seed=22, dtype=dtype)
        _announce("checkpoints", dtype.__name__, f64)
        ref = None
        for every in (1, 3, 7, 10):
            loss, gu, gp = _grad(model, 7, every, f64)
            if ref is None:
                ref = (loss, gu, gp)
            else:
                assert loss == ref[0] and np.array_equal(gu, ref[1]) and np.array_equal(gp, ref[2])


def _fd_ok(g, rows, slack=0.0):
    """D_K is piecewise linear with kinks at every scale along a generic
    direction: accept the adjoint value if, for some stored step size h, it
    matches the central difference, or lies between the two one-sided
    differences, within 1e-4 relative.  `slack` widens that interval by a
    multiple of the one-sided differences' own disagreement (used for dense
    directions, where at h = 1e-9 the FP64 rounding of D_K, about 1e-13 of
    its value, already moves a one-sided difference by ~1e-3)."""
    for r in rows:
        tol = 1e-4 * max(1.0, abs(r["central"])) + slack * abs(r["right"] - r["left"])
        lo, hi = min(r["left"], r["right"]), max(r["left"], r["right"])
        if abs(g - r["central"]) <= tol or lo - tol <= g <= hi + tol:
            return True
    return False


def test_fp32_adjoint_matches_stored_finite_differences_full_size():
    """The differentiation workload (n=100, L=32, K=50, checkpoints every 10)
    on an FP32 handle: loss and gradient (of the FP64 twin run, the default)
    against FP64 finite differences of the oracle along 8 dense and 8 sparse
    seeded directions and 24 coordinates."""
    import sys
    path = os.path.join(GOLD, "adjoint_uniform_k100_l32.json")
    g = json.load(open(path))
    sys.path.insert(0, GOLD)
    import make_golden as MG
    _announce("fp32 adjoint n=100 L=32 K=50")
    model = W.uniform(100, 32, seed=0)
    loss, gu, gp = _grad(model, g["K"], g["every"])
    assert abs(loss - g["D"]) <= 1e-5 * abs(g["D"])
    base = model.astype(np.float64)
    gu64, gp64 = gu.astype(np.float64), gp.astype(np.float64)
    bad = []
    for name, dirs in (("dense", MG.adjoint_directions(base, g["dense"]["count"], g["dense"]["seed"])),
                       ("sparse", MG.adjoint_sparse_directions(base, g["sparse"]["count"], g["sparse"]["seed"],
                                                               g["sparse"]["support"]))):
        for k, (du, dp) in enumerate(dirs):
            proj = float((gu64 * du).sum() + (gp64 * dp).sum())
            if not _fd_ok(proj, g[name]["fd"][k], 0.5 if name == "dense" else 0.0):
                bad.append((name, k, proj, g[name]["fd"][k]))
    flat = np.concatenate([gu64.ravel(), gp64.ravel()])
    assert g["coords"]["index"] == MG.adjoint_coords(base, g["coords"]["count"], g["coords"]["seed"])
    for k, c in enumerate(g["coords"]["index"]):
        if not _fd_ok(float(flat[c]), g["coords"]["fd"][k]):
            bad.append(("coord", c, float(flat[c]), g["coords"]["fd"][k]))
    assert not bad, bad


def test_fp32_run_adjoint_is_close_to_the_fp64_twin():
    """The gradient of the FP32 run itself (OPT_ADJOINT_F64 = 0) picks a
    neighbouring linear piece for the minimizers that FP32 rounding flips;
    it stays within a few percent of the FP64 twin's gradient, and its loss
    within 1e-5 of the oracle's."""
    path = os.path.join(GOLD, "adjoint_uniform_k100_l32.json")
    g = json.load(open(path))
    _announce("fp32-run adjoint vs fp64 twin")
    model = W.uniform(100, 32, seed=0)
    l32, gu32, gp32 = _grad(model, g["K"], g["every"], 0)
    l64, gu64, gp64 = _grad(model, g["K"], g["every"], 1)
    assert abs(l32 - g["D"]) <= 1e-5 * abs(g["D"])
    a = np.concatenate([gu32.ravel(), gp32.ravel()]).astype(np.float64)
    b = np.concatenate([gu64.ravel(), gp64.ravel()]).astype(np.float64)
    rel = np.linalg.norm(a - b) / np.linalg.norm(b)
    print("fp32-run vs fp64-twin gradient: rel L2", rel, "entries equal", float(np.mean(a == b)), flush=True)
    assert rel <= 3e-2


def test_orientation_and_degenerate_models():
    _announce("adjoint orientation/degenerate")
    model = W.uniform(7, 3, seed=23, dtype=np.float64)
    flip = W.Model(model.n, model.L, model.edges[:, ::-1].copy(), model.unaries,
                   np.transpose(model.pairwise, (0, 2, 1)).copy())
    la, gua, gpa = _grad(model, 4, 2)
    lb, gub, gpb = _grad(flip, 4, 2)
    assert la == lb and np.array_equal(gua, gub)
    assert np.array_equal(gpa, np.transpose(gpb, (0, 2, 1)))
    # no edges: D = sum_u min theta_u, gradient = one-hot at the smallest minimizer
    un = np.array([[0.5, 0.25, 0.25], [1.0, 2.0, 0.0]], np.float64)
    m0 = W.Model(2, 3, np.zeros((0, 2), np.int32), un, np.zeros((0, 3, 3)))
    loss, gu, gp = _grad(m0, 3, 2)
    assert loss == 0.25 and np.array_equal(gu, [[0, 1, 0], [0, 0, 1]])


def test_backward_requires_a_forward():
    _announce("adjoint state")
    model = W.uniform(6, 3, seed=24)
    with M.Solver.from_model(model) as s:
        with pytest.raises(M.MplpError) as ei:
            s.adjoint_backward()
        assert ei.value.code == M.ESTATE
        s.adjoint_forward(3, 1)
        s.iterate(1)
        with pytest.raises(M.MplpError) as ei:
            s.adjoint_backward()
        assert ei.value.code == M.ESTATE


def test_autograd_function():
    import torch
    from paper_2004_08227_amd.autograd import mplp_dual
    _announce("autograd")
    model = W.uniform(12, 5, seed=25)
    un = torch.tensor(model.unaries, device="cuda", requires_grad=True)
    pw = torch.tensor(model.pairwise, device="cuda", requires_grad=True)
    loss = mplp_dual(un, pw, model.edges, K=6, every=3)
    (2.0 * loss).backward()
    l2, gu, gp = _grad(model, 6, 3)
    assert float(loss.detach()) == np.float32(l2)
    assert np.array_equal(un.grad.cpu().numpy(), 2.0 * gu)
    assert np.array_equal(pw.grad.cpu().numpy(), 2.0 * gp)


def test_adjoint_memory_is_reported():
    """MPLPXX_INFO_ADJOINT_BYTES after a forward: checkpoints (K/every + 1
    copies of U and phi), one segment of argmin records (3 L bytes per edge
    and iteration), the adjoint buffers; an FP32 handle differentiating its
    FP64 twin adds the twin's costs and state."""
    _announce("adjoint bytes")
    n, L, K, every = 12, 5, 9, 4
    m64 = W.uniform(n, L, seed=3, dtype=np.float64)
    m = m64.m
    nck = (K + every - 1) // every
    nL, mp = n * L, m * 2 * L
    own64 = (nck + 1) * nL * 8 + (nck + 1) * mp * 8 + every * m * 3 * L + nL * 8 + mp * 8 + m * L * L * 8 + m * 8
    with M.Solver.from_model(m64) as s:
        assert s.info("adjoint_bytes") == 0
        s.adjoint_forward(K, every)
        assert s.info("adjoint_bytes") == own64
    m32 = W.uniform(n, L, seed=3, dtype=np.float32)
    with M.Solver.from_model(m32) as s:
        s.set_option(M.OPT_ADJOINT_F64, 1)
        s.adjoint_forward(K, every)
        twin = own64 + nL * 8 * 2 + m * L * L * 8 + mp * 8
        assert s.info("adjoint_bytes") == twin


@pytest.mark.parametrize("n,L,K", [(10, 64, 4), (8, 100, 3), (6, 128, 3)])
def test_fp64_adjoint_at_large_labels(n, L, K):
    """At L up to the library maximum (full and ragged tiles): adding c to
    every label of one node's unary, or to every entry of one edge's table,
    raises D_K by exactly c (the update (H) passes a uniform shift through
    and no argmin moves), so the gradient sums to 1 over each node's L
    entries and over each edge's L x L entries; and seeded coordinates match
    central differences of the oracle (a step may cross a kink of the
    piecewise-linear D_K for at most one of them)."""
    _announce("fp64 adjoint large L", n, L, K)
    model = W.uniform(n, L, seed=40 + L, dtype=np.float64)
    loss, gu, gp = _grad(model, K, 1)
    st, _ = oracle.run_model(model, K)
    assert abs(loss - st.dual()) <= 1e-12 * max(1, abs(loss))
    assert np.max(np.abs(gu.sum(axis=1) - 1.0)) <= 1e-9
    assert np.max(np.abs(gp.sum(axis=(1, 2)) - 1.0)) <= 1e-9
    rng = np.random.default_rng(L)
    bad = []
    for arr, g, count in ((model.unaries, gu, 8), (model.pairwise, gp, 8)):
        for _ in range(count):
            idx = tuple(int(rng.integers(0, d)) for d in arr.shape)
            du = np.zeros(model.unaries.shape)
            dp = np.zeros(model.pairwise.shape)
            (du if arr is model.unaries else dp)[idx] = 1.0
            fd = _fd(model, K, du, dp, 1e-7)
            if abs(g[idx] - fd) > 1e-6 * max(1.0, abs(fd)):
                bad.append((idx, float(g[idx]), fd))
    assert len(bad) <= 1, bad
